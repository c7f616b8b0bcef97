"""FP64 CPU oracle for the Ahmad-Cohen regular and irregular forces (test
infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never does, and this
package never imports the GPU library: the two share nothing but the seeded
input generators in ``workloads``.

The arithmetic lives in ``nb6_oracle.c`` (plain C, IEEE double); this module
only builds it with gcc and marshals numpy arrays through ctypes.
"""
from .oracle import (  # noqa: F401
    build,
    lib_path,
    predict,
    regular_force,
    pair_terms,
    irregular_force,
    regular_correct,
    max_threads,
    OracleResult,
    IrregularResult,
    CorrectResult,
)
