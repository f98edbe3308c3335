"""CPU oracle for RT-DetMCD -- TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 implementation of what the HIP library computes,
written from the paper (De Ketelaere, Hubert, Raymaekers, Rousseeuw, Vranckx,
"Real-time outlier detection for large datasets by RT-DetMCD", arXiv
1910.05615).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP path (``paper_1910_05615_amd``) and never imports it.

Parity status of each function is stated in its docstring; functions without a
pin say "parity unpinned".
"""
from .rtdetmcd import *  # noqa: F401,F403
from . import adjoint  # noqa: F401
