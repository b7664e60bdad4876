"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 definition of the particle costs, satisfaction mask,
gradient and Adam step.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does, and the oracle imports nothing from the HIP path (it reads only the
seeded input descriptors of ``paper_2411_11833_amd.inputs``).
"""
from .cutamp_oracle import *  # noqa: F401,F403
