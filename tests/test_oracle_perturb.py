"""Pins for the branching perturbation (Appendix D): mass, identity, structure."""
import math

import numpy as np

from oracle import lbm, perturb


def _state(seed):
    ch = lbm.Channel(40, 12, 0.55, 1e-5, (10, 4, 4))
    f = lbm.init_populations(ch, lbm.init_density(ch, seed, 0, 1e-2))
    f, _ = lbm.run(ch, f, 5)
    return ch, f


def test_mass_preserved_and_zero_eps_identity():
    ch, f = _state(1)
    fl = ~lbm.solid_mask(ch)
    snaps = np.stack([_state(s)[1] for s in range(2, 6)])
    al = perturb.alphas(key=3, slot=2, period=1, n_snap=4)
    g = perturb.perturb(f, snaps, al, 0.002, fl)
    assert math.isclose(perturb.total_mass(g, fl), perturb.total_mass(f, fl), rel_tol=2e-15)
    assert not np.allclose(g, f, rtol=0, atol=1e-7)
    assert np.array_equal(perturb.perturb(f, snaps, al, 0.0, fl), f)


def test_shift_is_a_positive_combination_then_one_scale():
    ch, f = _state(1)
    fl = ~lbm.solid_mask(ch)
    snaps = np.stack([_state(s)[1] for s in range(2, 5)])
    al = np.array([0.25, 0.5, 1.0])
    g = perturb.perturb(f, snaps, al, 0.01, fl)
    raw = f + 0.01 * (0.25 * snaps[0] + 0.5 * snaps[1] + 1.0 * snaps[2])
    ratio = g[:, fl] / raw[:, fl]
    assert np.allclose(ratio, ratio.flat[0], rtol=1e-14)
    assert ratio.flat[0] < 1  # positive snapshots add mass, the scale removes it


def test_alphas_uniform_and_distinct():
    a = np.concatenate([perturb.alphas(1, s, 0, 10) for s in range(400)])
    assert a.min() >= 0 and a.max() < 1
    assert abs(a.mean() - 0.5) < 0.02
    assert not np.array_equal(perturb.alphas(1, 0, 0, 10), perturb.alphas(1, 1, 0, 10))
    assert not np.array_equal(perturb.alphas(1, 0, 0, 10), perturb.alphas(1, 0, 1, 10))
