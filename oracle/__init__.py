"""CPU reference implementations (test infrastructure only).

Nothing in the product path may import, call or link anything in this
package: only the tests, the package's smoke check and the benchmark's CPU
baseline leg use it.  Everything here is plain NumPy/SciPy in float64,
written from the paper's definitions, and shares no code with the HIP
library.

Modules
  dense    O1: textbook CP-ALS on the explicitly formed order-4 tensor
           (tiny sizes only).  Fit by dense reconstruction.
  matfree  O2: the matrix-free THC-based CP-ALS of the paper (eq. lossF),
           in the same step order as the GPU path, any size.
  lt       Laplace-transform row scaling of the THC factors (eq. mp1_t and
           the THC-LT amplitude that follows it).
  warmstart  Warm-start features of the grid points, selection of the
           initial CP columns, training targets from converged CPDs.
  mlp      Warm-start network: forward, loss, manual backward, Adam.
  exchange Robust CPD+THC LT-MP2 exchange energy (single- and double-CPD
           terms, eq. rob_K).
  mp2      THC LT-MP2 Coulomb and exchange terms and the LT-MP2 energy.
  tied     Particle-tied CP-ALS (eq. cp4's one factor per particle) by
           symmetric ALS.
  df       Density-fitting tensors (eq. df_loss) and their exact THC form.
  order3   Order-3 THC-like tensors as the order-4 form with a singleton
           mode; the three-way CP-ALS they are pinned against.

Pins: every function is checked by ``tests/test_oracle_*.py`` against
brute-force loops, closed forms, planted decompositions, special cases and
invariances (see each module's header).  The paper prints no numeric
example for the CP-ALS itself, so there is no golden value from the paper.
"""
