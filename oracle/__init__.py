"""Plain FP64 CPU oracle of the cubic Fokker-Planck particle step.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py``.  It shares no code with the GPU library.
"""
