"""CPU FP64 oracle for the phonon BTE time step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library.
"""
from .oracle import Oracle, OracleError, build_oracle, oracle_lib_path  # noqa: F401
