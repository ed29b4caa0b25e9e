"""FP64 CPU oracle for the direct N-body force path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The oracle shares no code with the HIP
library and imports nothing from it.

The arithmetic lives in ``oracle.c`` (plain C, FP64 terms, long-double sums);
this module builds it with gcc, loads it with ctypes and adds the 4th-order
Hermite predictor-evaluator-corrector step used as a test harness (the paper
names 4th-order Hermite, Makino & Aarseth 1992, as its reference integrator in
the Results section; the library only supplies forces, the host integrator
does the correction).
"""

from .oracle import (  # noqa: F401
    build,
    lib_path,
    max_threads,
    predict,
    predict_jerk,
    force,
    force8,
    force_vjp,
    hermite4_correct,
    total_energy,
)
