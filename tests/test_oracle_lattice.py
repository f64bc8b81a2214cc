"""Pins of the oracle's lattice algebra (D3Q19 table, equilibrium, BGK + Guo
collision) against the definitions, not against the oracle itself.

The paper names no lattice or collision operator (sec. 2.3.2 only says
"LBM"); the reading is D3Q19 BGK with Guo forcing.  The pins are the
defining properties: the velocity set and weights of D3Q19, the exact
moments of the second-order equilibrium, and the moment-level effect of one
collision (mass kept, momentum raised by exactly F, second moment relaxed
by 1/tau plus the Guo source (1 - 1/(2 tau))(uF + Fu))."""
import itertools

import numpy as np
import pytest

import oracle


def d3q19_reference():
    """D3Q19 by definition: every e in {-1,0,1}^3 with |e|^2 <= 2; weights
    1/3, 1/18, 1/36 for |e|^2 = 0, 1, 2."""
    out = {}
    for e in itertools.product((-1, 0, 1), repeat=3):
        s = sum(x * x for x in e)
        if s <= 2:
            out[e] = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[s]
    return out


def test_table_is_d3q19():
    e, w, op = oracle.lattice()
    ref = d3q19_reference()
    assert len(ref) == 19
    got = {tuple(int(v) for v in e[i]): w[i] for i in range(19)}
    assert set(got) == set(ref)
    for k, v in ref.items():
        assert got[k] == pytest.approx(v, rel=0, abs=1e-17)
    for i in range(19):
        assert tuple(e[op[i]]) == tuple(-e[i])
    assert tuple(e[0]) == (0, 0, 0)


def test_weight_isotropy():
    e, w, _ = oracle.lattice()
    e = e.astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, e), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), np.eye(3) / 3, atol=1e-16)
    # fourth-order isotropy: sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso, atol=1e-16)


@pytest.mark.parametrize("rho,u", [(1.0, (0, 0, 0)), (1.03, (0.05, -0.02, 0.01)),
                                   (0.97, (-0.1, 0.07, 0.12))])
def test_equilibrium_moments(rho, u):
    e, _, _ = oracle.lattice()
    e = e.astype(float)
    u = np.array(u, float)
    f = oracle.feq(rho, u)
    assert f.sum() == pytest.approx(rho, abs=1e-14)
    assert np.allclose(e.T @ f, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("ia,ib,i->ab", e, e, f), rho * (np.outer(u, u) + np.eye(3) / 3),
                       atol=1e-15)


def _random_state(seed):
    rng = np.random.default_rng(seed)
    base = oracle.feq(1.0 + rng.uniform(-0.02, 0.02), rng.uniform(-0.05, 0.05, 3))
    return base * (1 + rng.uniform(-0.05, 0.05, 19))


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("tau", [0.55, 0.8, 1.3])
def test_collision_moments(seed, tau):
    """Mass kept; momentum raised by F = rho g; Pi+ = Pi - (Pi - Pi_eq)/tau
    + (1 - 1/(2 tau)) (u F + F u), with rho u = sum e f + F/2."""
    e, _, _ = oracle.lattice()
    e = e.astype(float)
    f = _random_state(seed)
    g = np.random.default_rng(100 + seed).uniform(-1e-3, 1e-3, 3)
    fp = oracle.collide_node(f, g, tau)
    rho = f.sum()
    F = rho * g
    u = (e.T @ f + F / 2) / rho
    assert fp.sum() == pytest.approx(rho, rel=1e-15)
    assert np.allclose(e.T @ fp, e.T @ f + F, atol=1e-15)
    Pi = np.einsum("ia,ib,i->ab", e, e, f)
    Pi_eq = rho * (np.outer(u, u) + np.eye(3) / 3)
    Pi_p = Pi - (Pi - Pi_eq) / tau + (1 - 0.5 / tau) * (np.outer(u, F) + np.outer(F, u))
    assert np.allclose(np.einsum("ia,ib,i->ab", e, e, fp), Pi_p, atol=1e-14)


def test_rest_state_is_fixed_point():
    f = oracle.feq(1.0, [0, 0, 0])
    assert np.abs(oracle.collide_node(f, [0, 0, 0], 0.8) - f).max() < 1e-16
