"""Pins of the oracle's decoder-parameter gradient of the summed reduced
energy (the potential loss of the unsupervised subspace construction,
Sec. 3.2), which the GPU's reverse pass is checked against.

The oracle applies the chain rule by hand.  The pins use other computations:
central finite differences of the oracle's own energy in sampled parameters
(energies only, no derivative code), a vanishing gradient at the rest state,
and pinned output rows that cannot move.
"""
import copy

import numpy as np
import pytest

from paper_2409_03807_amd import inputs as I


def _problem(bias_scale=0.3):
    return I.make_problem("pg", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=bias_scale)


def _summed_energy(O, p, z, tg, fo, flags):
    E, _, _ = O.Oracle(p).reduced(z, tg, fo, flags=O.ENERGY_ONLY | flags)
    return float(E.sum())


@pytest.mark.parametrize("flags", [0, 2])
def test_param_grad_matches_central_differences(oracle_mod, flags):
    O = oracle_mod
    p = _problem()
    B = 3
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    o = O.Oracle(p)
    E, grad = o.energy_param_grad(z, tg, fo, flags=flags)
    E_ref, _, _ = o.reduced(z, tg, fo, flags=O.ENERGY_ONLY | flags)
    np.testing.assert_allclose(E, E_ref, rtol=1e-12)
    parts = o.unpack_params(grad)
    rng = np.random.default_rng(11 + flags)
    nL = len(parts)
    free_rows = np.nonzero(np.repeat(p.pinned == 0, 3))[0]
    for l, (gW, gb) in enumerate(parts):
        scale = max(np.abs(gW).max(), np.abs(gb).max())
        assert scale > 0
        picks = []
        for _ in range(6):
            i = int(rng.choice(free_rows)) if l == nL - 1 else int(rng.integers(gW.shape[0]))
            picks.append(("W", (i, int(rng.integers(gW.shape[1])))))
        for _ in range(3):
            i = int(rng.choice(free_rows)) if l == nL - 1 else int(rng.integers(gb.size))
            picks.append(("b", (i,)))
        for kind, idx in picks:
            q = copy.deepcopy(p)
            arr = q.Ws[l] if kind == "W" else q.bs[l]
            h = 1e-5 * max(1.0, abs(arr[idx]))
            arr[idx] += h
            Ep = _summed_energy(O, q, z, tg, fo, flags)
            arr[idx] -= 2 * h
            Em = _summed_energy(O, q, z, tg, fo, flags)
            fd = (Ep - Em) / (2 * h)
            an = (gW if kind == "W" else gb)[idx]
            # central differences: O(h^2) truncation plus rounding of E / h
            assert abs(fd - an) <= 1e-6 * scale, (l, kind, idx, fd, an)


def test_param_grad_vanishes_at_rest_and_on_pinned_rows(oracle_mod):
    O = oracle_mod
    # zero biases and z = 0 decode to the rest shape: no elastic force anywhere
    p = _problem(bias_scale=0.0)
    o = O.Oracle(p)
    z0 = np.zeros((2, p.r))
    _, g0 = o.energy_param_grad(z0, flags=O.ELASTIC_ONLY)
    z = I.latent_batch(2, p.r)
    tg, fo = I.loads_for(p, 2)
    _, g = o.energy_param_grad(z, tg, fo)
    assert np.abs(g0).max() <= 1e-9 * np.abs(g).max()
    # rows of pinned vertices never move, so their output weights have no gradient
    gW, gb = o.unpack_params(g)[-1]
    pinned_rows = np.nonzero(np.repeat(p.pinned == 1, 3))[0]
    assert len(pinned_rows) > 0
    assert np.all(gW[pinned_rows] == 0.0) and np.all(gb[pinned_rows] == 0.0)


def test_param_grad_is_additive_over_items(oracle_mod):
    O = oracle_mod
    p = _problem()
    o = O.Oracle(p)
    z = I.latent_batch(4, p.r)
    tg, fo = I.loads_for(p, 4)
    _, g = o.energy_param_grad(z, tg, fo)
    _, ga = o.energy_param_grad(z[:1], tg[:1] if tg is not None else None, fo[:1] if fo is not None else None)
    _, gb = o.energy_param_grad(z[1:], tg[1:] if tg is not None else None, fo[1:] if fo is not None else None)
    np.testing.assert_allclose(ga + gb, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())
