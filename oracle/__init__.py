"""Plain FP64 CPU oracle of the dynamic-circuit tensor-network method.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything here; the
product path (``paper_2609_26516_amd``) never does, and the two share no code.

Modules
  statevector  brute-force 2^n amplitude vector simulation (Def. III.1-III.6),
               the exact reference for small circuits
  mps          MPS, layered gate operators, the compression step (Sec. III-C),
               measurement probability and collapse (Sec. IV-B1)
  ttn          tree tensor network (Sec. II-B): structure, canonical starting
               guess, the compression step as single-node sweeps over the
               tree, measurement and collapse (small n: environments by brute
               force on the statevector)
  dynamic      single-path (Alg. 1) and multi-path (Alg. 2) drivers over an
               MPS or a tree, chunk construction (Sec. IV-C), top-M retention
               and adaptive pruning, TVD (Sec. V-A)

Everything is complex128 / float64, written for checkability, not speed.
Pins: see tests/test_oracle_*.py.  Parity is unpinned by the paper only for
the truncated regime of the compression (no printed values exist there); it
is pinned by closed forms, brute force and the Eckart-Young bound instead.
"""
