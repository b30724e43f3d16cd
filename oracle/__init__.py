"""FP64 CPU oracle of the coupled Yee-FDTD / kinetic plasma model (arXiv 2211.05647).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``, never by the product package.  It shares no code
with the HIP library.
"""
