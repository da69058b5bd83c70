"""CPU oracle for the loop-erased-walk estimators of arXiv 2311.10290.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  It shares no code with the HIP library in ``paper_2311_10290_amd``
and never imports it; the two meet only in the seeded inputs of
``graphgen``.

Contents
  native      -- builds and binds ``sampler.c``: scalar Wilson sampler with
                 stack-keyed Philox4x64-10 draws, v-absorbed walks,
                 loop-included paths (Sec. 3.4; Alg. 2; Alg. 4)
  csr         -- edge list -> simple connected CSR graph, landmark choice
  dense       -- FP64 dense ground truth: L^dagger by two routes, L_v^{-1},
                 (I-P_v)^{-1}, closeness, Kemeny's constant, resistance,
                 the identities of Thm. 1 and the element-wise equations
  estimators  -- FP64 assembly of the estimators from integer counts
                 (Alg. 2 last loop, Alg. 4 update, closeness formula)
  trees       -- brute-force spanning-tree enumeration for tiny graphs

Parity status: every function is pinned by tests under ``tests/`` that check
it against closed forms, the paper's worked examples, a library routine or
brute force.  ``estimators.rw_betweenness`` implements the formula quoted at
the end of Sec. 5 as printed; it is pinned by the closed forms on complete
graphs and stars and by the same quantity rebuilt from pairwise resistances.
"""
