"""The counter-based generator against its published definition and the recipe."""
import json
import os

import numpy as np

import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    out = synthetic.splitmix64(np.array(g["state_before_increment"], dtype=np.uint64))
    assert ["%016x" % int(x) for x in out] == g["output_hex"]


def test_uniform_and_gaussian_moments():
    u = synthetic.uniform(7, 1, np.arange(200000))
    assert 0.0 <= u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3
    z = synthetic.gaussian(7, 1, np.arange(200000))
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1.0) < 1e-2


def test_recipe_shapes_and_symmetries():
    o, v, n, seed = 3, 5, 7, 1
    Lvv = synthetic.draw_L_vv(seed, o, v, n)
    assert Lvv.shape == (v, v, n)
    assert np.array_equal(Lvv, Lvv.transpose(1, 0, 2))          # L^J_ac = L^J_ca
    full = synthetic.draw_L_block(seed, o + v, n, 0, o + v, 0, o + v)
    assert np.array_equal(full[o:, o:], Lvv)
    assert np.array_equal(full[:o, o:], synthetic.draw_L_ov(seed, o, v, n))
    eps = synthetic.draw_eps(seed, o, v)
    assert (eps[:o] >= -1.5).all() and (eps[:o] < -0.3).all()
    assert (eps[o:] >= 0.1).all() and (eps[o:] < 3.0).all()
    xi = synthetic.draw_noise_full(seed, o, v)
    assert np.array_equal(xi, xi.transpose(1, 0, 3, 2))          # xi_ij^ab = xi_ji^ba
    sizes = synthetic.batched_sizes(4, 64)
    assert len(sizes) == 64
    assert all(8 <= a <= 40 and 60 <= b <= 300 and c == 4 * (a + b) for a, b, c in sizes)
