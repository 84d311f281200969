"""CPU oracle for edge subdivision -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never does, and this
package never imports the GPU library: the two share no code.
"""
from .oracle import (  # noqa: F401
    OracleError,
    OracleResult,
    build,
    extract,
    extract_simplex,
    forward,
    vertex_solve,
)
