"""Oracle for the hardware-fitted linear run-time model.

TEST INFRASTRUCTURE ONLY.  Only tests/, `__graft_entry__.smoke()` and the
CPU-baseline leg of bench.py import this package.  It shares no code with
the HIP library under paper_1604_04997_amd/ and never imports it.

  count.py    simulated-execution counter (C, count_oracle.c) over every
              kernel family: the kernel properties of Sec. 2, counted as in
              Alg. 1 (Eq. opcount) with per-array footprints of Alg. 2
  outputs.py  plain NumPy / C references of every kernel's output
  model.py    derived features, the relative-error least-squares fit of
              Sec. 4.3 and the geometric-mean error of Sec. 5

Every function is pinned by tests that do not call the oracle's own
formulas again (closed forms, hand-enumerated tiny domains, the paper's
textbook stride classes and its Table 1 worked example); see tests/.
"""
