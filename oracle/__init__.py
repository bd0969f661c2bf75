"""FP64 CPU oracle for the SMPC plan step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  It shares no code with the HIP library
and is never on the product path.
"""
from . import edt, rng, smpc_oracle  # noqa: F401
