"""FP64 CPU oracle for the 3D fast super-resolution solvers.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
NumPy/SciPy restatement of what the GPU path computes, used to check it.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it. The HIP library and its Python binding never
import, call or link anything here, and nothing here imports them.
"""

from .sr3d_oracle import *  # noqa: F401,F403
