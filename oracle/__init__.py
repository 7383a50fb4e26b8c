"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package. The product path (``paper_2208_12569_amd``) never does, and the two share
no code: the only common dependency is the input generator package ``synth``.
"""

from .oracle import (  # noqa: F401
    ORC_OK,
    ORC_OUTSIDE,
    ORC_NULLB,
    ORC_MAXSTEPS,
    ORC_NONFINITE,
    ORC_ONESIDED,
    ORC_MIXEDFACE,
    ORC_EDGE,
    ORC_ROTATED,
    FATAL,
    build,
    curl,
    interp,
    trace,
    q2d,
    q3d,
    default_opts,
    threads,
    q2d_points,
    q3d_points,
    method2,
    q2d_perp,
    qcyl,
    ORC_FACE_CYL,
)
