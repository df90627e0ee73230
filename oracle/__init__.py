"""FP64 CPU oracle: plain, slow, obviously correct.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
The HIP library and its Python binding never do: the product path fails when
its compiled extension is missing instead of falling back to anything here.
"""
