"""FP64 CPU oracle for multislice STEM and PRISM.

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``,
and by nothing else. It shares no code with the HIP library; both only
consume the seeded inputs of the ``synth`` package.
"""
from .prism_oracle import *  # noqa: F401,F403
from .prism_oracle import __all__  # noqa: F401
