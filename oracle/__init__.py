"""Plain FP64 CPU oracle of the chi0 -> E_c path.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py may import it.  It shares no code with the GPU library
(paper_2407_19930_amd) and the library never imports it.

Modules:
  chi0        plain supercell definition, Algorithm 1, brute-force four-term sum
  aw          sum-over-states chi0 in tau and i omega
  transforms  cosine and R -> q transforms
  energy      E_c by LU log-determinant (and an eigenvalue route)
  pipeline    chi0(R, tau) -> E_c for a whole input bundle

Every function has a pin in tests/test_oracle_*.py that does not re-derive it:
closed forms, identities between independent routes, sign and symmetry
properties, and literal brute force on micro inputs.
"""
