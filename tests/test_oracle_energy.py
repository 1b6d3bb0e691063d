"""Pins of the oracle's energy and gradient against closed forms, finite
differences, an autograd formulation, invariances and exclusion rules
(section 2 of the paper)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from tests.systems import dihedral_points, make_system, random_rotation, torsion_chain

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_coulomb_constant_fixture(golden):
    c = golden["coulomb_constant"]
    from synth import COULOMB_KCAL
    assert c["paper_kj"] == 1389.38757
    assert COULOMB_KCAL == pytest.approx(c["paper_kj"] / c["kj_per_kcal"], rel=0, abs=0)
    assert COULOMB_KCAL == pytest.approx(c["kcal_value"], rel=1e-15)


# ---------------------------------------------------------------- P1-P3 pairs

@pytest.mark.parametrize("sig,eps", [(3.0, 0.1), (3.7, 0.17)])
def test_lj_minimum_closed_form(golden, sig, eps):
    rstar = golden["lj"]["r_min_over_sigma"] * sig
    s = make_system([[0, 0, 0], [rstar, 0, 0]], sigma=[sig, sig], eps=[eps, eps])
    terms, g = oracle.energy_terms(s, s["x"])
    assert terms["vdw"] == pytest.approx(-eps, rel=1e-12)
    assert terms["coulomb"] == 0.0
    assert np.abs(g).max() < 1e-12 * eps / sig * 100
    # energy at r = sigma is exactly zero, at 2^(1/6) sigma it is the minimum
    s2 = make_system([[0, 0, 0], [0, sig, 0]], sigma=[sig, sig], eps=[eps, eps])
    assert abs(oracle.energy_terms(s2, s2["x"])[0]["vdw"]) < 1e-13


def test_lj_curve_and_force():
    sig, eps = 3.3, 0.12
    for r in (2.5, 3.0, 3.7, 5.0, 11.0):
        s = make_system([[0, 0, 0], [0, 0, r]], sigma=[sig, sig], eps=[eps, eps])
        terms, g = oracle.energy_terms(s, s["x"])
        e = 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)
        dedr = 4 * eps * (-12 * sig ** 12 / r ** 13 + 6 * sig ** 6 / r ** 7)
        assert terms["vdw"] == pytest.approx(e, rel=1e-13)
        # atom 1 sits at +z: dE/dz_1 = dE/dr, dE/dz_0 = -dE/dr
        assert g[1, 2] == pytest.approx(dedr, rel=1e-12)
        assert g[0, 2] == pytest.approx(-dedr, rel=1e-12)
        assert np.abs(g[:, :2]).max() == 0.0


def test_coulomb_pair():
    from synth import COULOMB_KCAL
    q1, q2, r = 0.4, -0.3, 4.2
    s = make_system([[1, 2, 3], [1 + r, 2, 3]], q=[q1, q2], eps=[0, 0])
    terms, g = oracle.energy_terms(s, s["x"])
    assert terms["vdw"] == 0.0
    assert terms["coulomb"] == pytest.approx(COULOMB_KCAL * q1 * q2 / r, rel=1e-14)
    assert np.linalg.norm(g[0]) == pytest.approx(COULOMB_KCAL * abs(q1 * q2) / r ** 2, rel=1e-14)
    # opposite charges attract: the gradient on atom 0 (at smaller x) points
    # away from atom 1, i.e. towards -x
    assert g[0, 0] < 0 and g[1, 0] > 0


def test_geometric_mixing():
    s1, e1, s2, e2, r = 3.1, 0.07, 3.9, 0.19, 4.0
    s = make_system([[0, 0, 0], [r, 0, 0]], sigma=[s1, s2], eps=[e1, e2])
    terms, _ = oracle.energy_terms(s, s["x"])
    sm, em = math.sqrt(s1 * s2), math.sqrt(e1 * e2)
    assert terms["vdw"] == pytest.approx(4 * em * ((sm / r) ** 12 - (sm / r) ** 6), rel=1e-14)


# ---------------------------------------------------------------- P4-P7 bonded

def test_bond_closed_form_and_exclusion():
    K, r0, r = 300.0, 1.5, 1.62
    s = make_system([[0, 0, 0], [0, r, 0]], q=[0.5, -0.5], eps=[0.2, 0.2],
                    bonds=[[0, 1]], bond_k=[K], bond_r0=[r0])
    terms, g = oracle.energy_terms(s, s["x"])
    assert terms["coulomb"] == 0.0 and terms["vdw"] == 0.0       # the 1-2 pair is excluded
    assert terms["stretch"] == pytest.approx(K * (r - r0) ** 2, rel=1e-14)
    assert g[1, 1] == pytest.approx(2 * K * (r - r0), rel=1e-14)
    s["x"] = np.array([[0, 0, 0], [0, r0, 0]])
    terms, g = oracle.energy_terms(s, s["x"])
    assert terms["stretch"] == 0.0 and np.abs(g).max() == 0.0


@pytest.mark.parametrize("theta_deg", [95.0, 109.5, 130.0])
def test_angle_closed_form(theta_deg):
    K, t0 = 50.0, math.radians(109.5)
    th = math.radians(theta_deg)
    x = [[1.4, 0, 0], [0, 0, 0], [1.6 * math.cos(th), 1.6 * math.sin(th), 0]]
    s = make_system(x, q=[0.3, 0.1, -0.4], eps=[0.1] * 3, angles=[[0, 1, 2]], angle_k=[K],
                    angle_t0=[t0], bonds=[[0, 1], [1, 2]], bond_k=[0, 0], bond_r0=[1.4, 1.6])
    terms, g = oracle.energy_terms(s, s["x"])
    assert terms["coulomb"] == 0.0 and terms["vdw"] == 0.0       # 1-2 and 1-3 excluded
    assert terms["bend"] == pytest.approx(K * (th - t0) ** 2, rel=1e-12, abs=1e-14)
    if theta_deg == 109.5:
        assert np.abs(g).max() < 1e-12
    else:
        # the force on the outer atom is tangential: magnitude 2K(th-t0)/|u|
        assert np.linalg.norm(g[0]) == pytest.approx(2 * K * abs(th - t0) / 1.4, rel=1e-12)
        assert abs(np.dot(g[0], np.array(x[0]))) < 1e-10


@pytest.mark.parametrize("phi_deg,expect", [(0.0, "v1+v3"), (180.0, "zero"), (90.0, "half"),
                                            (-90.0, "half")])
def test_torsion_special_angles(phi_deg, expect):
    V = [1.3, -0.7, 0.45, 0.2]
    x = dihedral_points(math.radians(phi_deg))
    s = make_system(x, dihedrals=[[0, 1, 2, 3]], dihedral_v=[V])
    terms, _ = oracle.energy_terms(s, s["x"])
    want = {"v1+v3": V[0] + V[2], "zero": 0.0, "half": 0.5 * V[0] + V[1] + 0.5 * V[2]}[expect]
    assert terms["torsion"] == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_exclusion_sets():
    # 3-atom chain: only bonded terms; 4-atom chain: exactly the (0,3) pair
    x3 = [[0, 0, 0], [1.5, 0, 0], [2.0, 1.4, 0]]
    kw = dict(q=[0.3, -0.2, 0.4], sigma=[3.2, 3.4, 3.6], eps=[0.1, 0.12, 0.15],
              bonds=[[0, 1], [1, 2]], bond_k=[0, 0], bond_r0=[1.5, 1.5],
              angles=[[0, 1, 2]], angle_k=[0], angle_t0=[1.9])
    t3, _ = oracle.energy_terms(make_system(x3, **kw), x3)
    assert t3["coulomb"] == 0.0 and t3["vdw"] == 0.0
    x4 = x3 + [[3.5, 1.0, 1.2]]
    kw4 = dict(q=[0.3, -0.2, 0.4, -0.25], sigma=[3.2, 3.4, 3.6, 3.0], eps=[0.1, 0.12, 0.15, 0.08],
               bonds=[[0, 1], [1, 2], [2, 3]], bond_k=[0, 0, 0], bond_r0=[1.5] * 3,
               angles=[[0, 1, 2], [1, 2, 3]], angle_k=[0, 0], angle_t0=[1.9, 1.9])
    s4 = make_system(x4, **kw4)
    t4, _ = oracle.energy_terms(s4, x4)
    pair = make_system([x4[0], x4[3]], q=[0.3, -0.25], sigma=[3.2, 3.0], eps=[0.1, 0.08])
    tp, _ = oracle.energy_terms(pair, pair["x"])
    assert t4["coulomb"] == pytest.approx(tp["coulomb"], rel=1e-15)
    assert t4["vdw"] == pytest.approx(tp["vdw"], rel=1e-15)


# ------------------------------------------------------------------ P8 FD

@pytest.mark.parametrize("seed", [3, 4])
def test_gradient_central_differences(seed):
    s = torsion_chain(24, seed)
    x = s["x"].copy()
    e0, g = oracle.energy_grad(s, x)
    h = 1e-5
    num = np.zeros_like(g)
    for i in range(x.shape[0]):
        for c in range(3):
            xp = x.copy(); xp[i, c] += h
            xm = x.copy(); xm[i, c] -= h
            num[i, c] = (oracle.energy_grad(s, xp, False)[0] - oracle.energy_grad(s, xm, False)[0]) / (2 * h)
    big = np.abs(g) > 1e-3
    rel = np.abs(num - g)[big] / np.abs(g)[big]
    assert rel.max() < 1e-6, rel.max()
    if (~big).any():
        assert np.abs(num - g)[~big].max() < 1e-8


def test_each_term_gradient_by_differences():
    s = torsion_chain(12, 7)
    x = s["x"].copy()
    rng = np.random.default_rng(0)
    x += rng.normal(scale=0.05, size=x.shape)
    # switch terms on one at a time via parameter masks
    masks = {
        "stretch": dict(angle_k=0, dihedral_v=0, q=0, eps=0),
        "bend": dict(bond_k=0, dihedral_v=0, q=0, eps=0),
        "torsion": dict(bond_k=0, angle_k=0, q=0, eps=0),
        "coulomb": dict(bond_k=0, angle_k=0, dihedral_v=0, eps=0),
        "vdw": dict(bond_k=0, angle_k=0, dihedral_v=0, q=0),
    }
    for name, zero in masks.items():
        t = dict(s)
        for k in zero:
            t[k] = np.zeros_like(np.asarray(s[k], float))
        _, g = oracle.energy_grad(t, x)
        h = 1e-5
        for i in (0, 5, 11):
            for c in range(3):
                xp = x.copy(); xp[i, c] += h
                xm = x.copy(); xm[i, c] -= h
                d = (oracle.energy_terms(t, xp, False)[0][name] - oracle.energy_terms(t, xm, False)[0][name]) / (2 * h)
                assert d == pytest.approx(g[i, c], rel=1e-6, abs=1e-7), (name, i, c)


# -------------------------------------------------------------- P9 invariances

def test_net_force_torque_and_rigid_motion():
    from synth import chain_system
    s = chain_system(300, 11)
    x = s["x"]
    e, g = oracle.energy_grad(s, x)
    scale = np.abs(g).sum()
    assert np.abs(g.sum(axis=0)).max() < 1e-10 * scale
    assert np.abs(np.cross(x, g).sum(axis=0)).max() < 1e-10 * scale * np.abs(x).max()
    rng = np.random.default_rng(5)
    R = random_rotation(rng)
    t = rng.normal(size=3) * 10
    e2, g2 = oracle.energy_grad(s, x @ R.T + t)
    assert e2 == pytest.approx(e, rel=1e-10)
    assert np.abs(g2 - g @ R.T).max() < 1e-10 * np.abs(g).max()


# ------------------------------------------------------ P10 autograd, tiny N

def _torch_energy(s, x):
    import torch
    X = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    n = s["n_atoms"]
    E = torch.zeros((), dtype=torch.float64)
    for (i, j), k, r0 in zip(s["bonds"], s["bond_k"], s["bond_r0"]):
        E = E + k * (torch.linalg.norm(X[i] - X[j]) - r0) ** 2
    for (i, j, k), kt, t0 in zip(s["angles"], s["angle_k"], s["angle_t0"]):
        u, v = X[i] - X[j], X[k] - X[j]
        th = torch.acos(torch.dot(u, v) / (torch.linalg.norm(u) * torch.linalg.norm(v)))
        E = E + kt * (th - t0) ** 2
    for (a, b, c, d), V in zip(s["dihedrals"], s["dihedral_v"]):
        b1, b2, b3 = X[b] - X[a], X[c] - X[b], X[d] - X[c]
        n1, n2 = torch.linalg.cross(b1, b2), torch.linalg.cross(b2, b3)
        m1 = torch.linalg.cross(n1, b2 / torch.linalg.norm(b2))
        phi = torch.atan2(torch.dot(m1, n2), torch.dot(n1, n2))
        E = E + 0.5 * (V[0] * (1 + torch.cos(phi)) + V[1] * (1 - torch.cos(2 * phi))
                       + V[2] * (1 + torch.cos(3 * phi)) + V[3] * (1 - torch.cos(4 * phi)))
    excl = {tuple(sorted(map(int, b))) for b in s["bonds"]}
    excl |= {tuple(sorted((int(a[0]), int(a[2])))) for a in s["angles"]}
    for i in range(n):
        for j in range(i + 1, n):
            if (i, j) in excl:
                continue
            r = torch.linalg.norm(X[i] - X[j])
            E = E + s["coulomb_c"] * s["q"][i] * s["q"][j] / r
            sg = math.sqrt(s["sigma"][i] * s["sigma"][j])
            ep = math.sqrt(s["eps"][i] * s["eps"][j])
            E = E + 4 * ep * ((sg / r) ** 12 - (sg / r) ** 6)
    E.backward()
    return float(E), X.grad.numpy()


@pytest.mark.parametrize("seed", [1, 2])
def test_autograd_tiny(seed):
    s = torsion_chain(9, seed)
    x = s["x"] + np.random.default_rng(seed).normal(scale=0.1, size=s["x"].shape)
    e, g = oracle.energy_grad(s, x)
    et, gt = _torch_energy(s, x)
    assert e == pytest.approx(et, rel=1e-12)
    assert np.abs(g - gt).max() < 1e-12 * max(1.0, np.abs(gt).max())


def test_atom_gradients_match_full():
    from synth import chain_system
    s = chain_system(200, 9)
    s2 = torsion_chain(200, 9)
    for sysd in (s, s2):
        _, g = oracle.energy_grad(sysd, sysd["x"])
        atoms = [0, 1, 57, 198, 199]
        ga = oracle.atom_gradients(sysd, sysd["x"], atoms)
        assert np.abs(ga - g[atoms]).max() <= 1e-12 * np.abs(g).max()


def test_bad_index_rejected():
    s = make_system([[0, 0, 0], [1, 0, 0]], bonds=[[0, 2]], bond_k=[1], bond_r0=[1])
    with pytest.raises(ValueError):
        oracle.energy_grad(s, s["x"])


# ------------------------------------------------ energy profile (section 3)

@pytest.mark.parametrize("r0", [2.8, 3.2, 4.5])
def test_profile_of_two_atoms_is_the_lj_curve(r0):
    """Two LJ atoms on the x axis: the unit antigradient moves each one by
    t/sqrt(2) along the axis, so the separation is r0 + sqrt(2) t on the
    repulsive side (r0 < 2^(1/6) sigma) and r0 - sqrt(2) t on the attractive
    one."""
    sig, eps = 3.4, 0.2
    s = make_system([[0, 0, 0], [r0, 0, 0]], sigma=[sig, sig], eps=[eps, eps])
    t = np.array([-0.3, 0.0, 0.05, 0.2, 0.7])
    e = oracle.energy_profile(s, s["x"], t)
    sign = 1.0 if r0 < 2 ** (1 / 6) * sig else -1.0
    r = r0 + sign * math.sqrt(2.0) * t
    lj = 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)
    np.testing.assert_allclose(e, lj, rtol=1e-12)


def test_profile_slope_at_zero_is_minus_the_gradient_norm():
    s = torsion_chain(40, 3)
    _, g = oracle.energy_grad(s, s["x"])
    h = 1e-5
    e = oracle.energy_profile(s, s["x"], [-h, 0.0, h])
    assert (e[2] - e[0]) / (2 * h) == pytest.approx(-np.linalg.norm(g), rel=1e-6)
    assert e[1] == pytest.approx(oracle.energy_grad(s, s["x"])[0], rel=1e-15)


def test_profile_with_a_zero_gradient_stays_put():
    s = make_system([[1.0, 2.0, 3.0]], sigma=[3.0], eps=[0.2], q=[0.4])
    np.testing.assert_array_equal(oracle.energy_profile(s, s["x"], [-1.0, 0.0, 2.5]), np.zeros(3))
