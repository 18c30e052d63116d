"""Plain, slow CPU oracle for the hard-to-round (HR) case search.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.
The oracle shares no code with the HIP path (no kernels, headers, helpers,
tables or constants).  It is written from the paper (Fortin, Gouicem,
Graillat, "GPU-accelerated generation of correctly-rounded elementary
functions") and each function cites the passage it follows.

Modules
  cf        continued fractions and two-length configurations (Sec. 3.2,
            Table 2, Fig. 3, Eq. 2/3, Props. 1-2)
  search    brute-force degree-1 hit lists (the definition behind Eq. 1) and
            the paper's lower-bound tests (Alg. 1, 2, 4)
  tabulate  straightforward shift (Sec. 5.2) and tabulated differences
            (Sec. 5.2, Fig. 7) over exact W-bit fixed point
  taylor    Taylor polynomials, Newton/hierarchical initial tables
            (Sec. 5.1, Fig. 6) and error bounds
  hr        per-argument brute force HR cases (Def. 2-3) and the three-phase
            pipeline oracle (Sec. 4.1)
  native    ctypes loader for the C part of the oracle (brute force and the
            exhaustive phase), compiled from oracle/c/hr_oracle.c

Every function is pinned by tests under ``tests/test_oracle_*.py`` except
where its header says "parity unpinned".
"""
