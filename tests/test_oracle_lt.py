"""Pin for oracle/lt.py: scaled THC factors give the denominator-weighted tensor."""
import numpy as np

from oracle import dense, lt
from synth import make_lt_system


def test_lt_scaling_is_denominator_weighting():
    Xo, Xv, Z, eo, ev = make_lt_system(3, 5, 0, rank_factor=2)
    t = 0.7
    base = dense.dense_tensor([Xo, Xv, Xo, Xv], Z)
    scaled = dense.dense_tensor(lt.lt_factors(Xo, Xv, eo, ev, t), Z)
    D = (ev[None, :, None, None] + ev[None, None, None, :]
         - eo[:, None, None, None] - eo[None, None, :, None])
    np.testing.assert_allclose(scaled, np.exp(-D * t) * base, rtol=1e-13, atol=1e-300)
