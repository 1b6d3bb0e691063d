"""GPU parity of the learned-warm-start kernels against the numpy oracle,
through the C ABI.

Bars: features, neighbour lists, conversions, gathers, selections and
integer-valued products are bit-exact.  The network compares with the
oracle's BF16 emulation: both round the same operands to BF16, but the GPU
accumulates in FP32 in another order, so a rounded activation can land on
the neighbouring BF16 value (one unit in the last place, at most 2^-7
relative).  The forward test bounds each output by 2^-6 times the absolute
products through which such a flip could reach it; on random inputs the
gradients are compared per parameter block in relative 2-norm against BF16's
unit roundoff 2^-8, and on inputs where every rounding and sum is exact
(tests/learn_exact.py) the forward output and every gradient element must
equal the oracle's.
"""
import numpy as np
import pytest
import torch

from oracle import learn as OL
from paper_1810_03358_amd import learn as L
from synth import chain_system
from tests.systems import make_system

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _systems():
    line = make_system(np.stack([np.arange(30.0), np.zeros(30), np.zeros(30)], axis=1),
                       q=np.linspace(-0.4, 0.4, 30), sigma=np.full(30, 3.3), eps=np.full(30, 0.1))
    lone = make_system([[1.0, 2.0, 3.0]], q=[0.2], sigma=[3.7], eps=[0.15])
    return [chain_system(300, 1), chain_system(10, 2), line, chain_system(17, 3), lone, chain_system(65, 4)]


def _features_gpu(systems):
    sa = L.SystemArrays(systems, DEV)
    x = torch.tensor(np.concatenate([s["x"] for s in systems]), dtype=torch.float64, device=DEV).contiguous()
    f, nb = L.features(sa, x, want_neighbors=True)
    return sa, x, f.cpu().numpy().view(np.uint16), nb.cpu().numpy()


def _oracle_inputs(systems):
    cat = lambda k: np.concatenate([np.asarray(s[k], dtype=np.float64) for s in systems])
    return np.concatenate([s["x"] for s in systems]), cat("q"), cat("sigma"), cat("eps")


def test_features_are_bit_exact():
    systems = _systems()
    sa, _, f, nb = _features_gpu(systems)
    x, q, s, e = _oracle_inputs(systems)
    fo, nbo = OL.features(x, q, s, e, sa.sys_first_host)
    np.testing.assert_array_equal(nb, nbo)
    np.testing.assert_array_equal(f, fo)


def test_features_at_10k_atoms_on_sampled_rows():
    systems = [chain_system(10_000, 1)]
    sa, _, f, nb = _features_gpu(systems)
    x, q, s, e = _oracle_inputs(systems)
    rows = np.random.default_rng(0).choice(10_000, size=150, replace=False)
    fo, nbo = OL.features(x, q, s, e, sa.sys_first_host, rows=rows)
    np.testing.assert_array_equal(nb[rows], nbo)
    np.testing.assert_array_equal(f[rows], fo)


def _bf16_dev(a):
    return torch.tensor(OL.bf16_bits(a).view(np.int16), device=DEV)


@pytest.mark.parametrize("m,n,k,trans_a,trans_b", [
    (1, 1, 1, False, False), (17, 33, 45, False, False), (130, 16, 128, True, False),
    (64, 128, 4099, True, False), (300, 128, 16, False, True), (16, 16, 16, True, True),
    # the LDS-tiled kernel (blocks of 64 x 64 x 32): every layout, ragged edges,
    # strides that do and do not allow 16-byte loads
    (64, 64, 32, False, False), (200, 128, 128, False, False), (64, 128, 300, True, False),
    (256, 64, 96, False, True), (129, 192, 70, True, True), (1000, 128, 45, False, False)])
def test_gemm_is_exact_on_small_integers(m, n, k, trans_a, trans_b):
    """Integer operands in [-8, 8]: every product and partial sum is exact in
    FP32 (|sum| <= 64 k < 2^24), so any accumulation order gives the same C."""
    rng = np.random.default_rng(m * 1000 + n + k)
    A = rng.integers(-8, 9, size=(m, k)).astype(np.float64)
    B = rng.integers(-8, 9, size=(k, n)).astype(np.float64)
    a_store = A.T.copy() if trans_a else A
    b_store = B.T.copy() if trans_b else B
    sa = (1, m) if trans_a else (k, 1)
    sb = (1, k) if trans_b else (n, 1)
    bias = rng.integers(-4, 5, size=n).astype(np.float32)
    c = torch.full((m, n), np.nan, dtype=torch.float32, device=DEV)
    cb = torch.zeros((m, n), dtype=torch.int16, device=DEV)
    L.gemm(_bf16_dev(a_store), sa, _bf16_dev(b_store), sb, m, n, k, out=c)
    np.testing.assert_array_equal(c.cpu().numpy(), A @ B)
    L.gemm(_bf16_dev(a_store), sa, _bf16_dev(b_store), sb, m, n, k,
           bias=torch.tensor(bias, device=DEV), relu=True, out=c, out_bf16=cb)
    want = np.maximum(A @ B + bias, 0.0)
    np.testing.assert_array_equal(c.cpu().numpy(), want)
    np.testing.assert_array_equal(cb.cpu().numpy().view(np.uint16), OL.bf16_bits(want))


def _theta(seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.normal(scale=0.125, size=128 * 128), rng.normal(scale=0.05, size=128),
                           rng.normal(scale=0.125, size=128 * 128), rng.normal(scale=0.05, size=128),
                           rng.normal(scale=0.1, size=128 * 16), rng.normal(scale=0.05, size=16)]).astype(np.float32)


def _chain_rows(n_rows, seed):
    systems = [chain_system(n_rows, seed)]
    sa, x, f, _ = _features_gpu(systems)
    return f


@pytest.mark.parametrize("rows", [1, 77, 1000, 4096])
def test_forward_matches_the_oracle(rows):
    theta = _theta(rows)
    fbits = _chain_rows(max(rows, 20), rows)[:rows]
    net = L.Net(theta, device=DEV)
    y = net.forward(torch.tensor(fbits.view(np.int16), device=DEV)).cpu().numpy().astype(np.float64)
    X = OL.bf16_value(fbits)
    yo, c = OL.forward(theta.astype(np.float64), X, emulate=True)
    bound = 2.0 ** -6 * (np.abs(c["H2r"]) @ np.abs(c["W3"]) + (np.abs(c["H1r"]) @ np.abs(c["W2"])) @ np.abs(c["W3"]))
    # FP32 accumulation of the first layer near a ReLU kink, and of the others
    P = {k: np.abs(v).astype(np.float64) for k, v in OL.unpack(theta).items()}
    bound += 2.0 ** -14 * (((np.abs(X) @ P["W1"] + P["b1"]) @ P["W2"] + P["b2"]) @ P["W3"] + P["b3"])
    assert np.all(np.abs(y - yo) <= bound)
    # flips are rare: a row of 256 rounded activations holds one with a
    # probability of a few percent; the other rows agree to FP32 accuracy
    close = np.all(np.abs(y - yo) <= 1e-5 * (np.abs(c["H2r"]) @ np.abs(c["W3"]) + 1e-30), axis=1)
    assert close.mean() >= 0.9


@pytest.mark.parametrize("rows", [33, 2048])
def test_backward_matches_the_oracle(rows):
    theta = _theta(100 + rows)
    fbits = _chain_rows(max(rows, 40), rows)[:rows]
    T = np.random.default_rng(rows).normal(scale=0.3, size=(rows, 3)).astype(np.float32)
    net = L.Net(theta, device=DEV)
    loss = net.loss_grad(torch.tensor(fbits.view(np.int16), device=DEV), torch.tensor(T, device=DEV))
    g = net.grad.cpu().numpy().astype(np.float64)
    lo, go = OL.loss_grad(theta.astype(np.float64), OL.bf16_value(fbits), T.astype(np.float64), emulate=True)
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=2.0 ** -8)
    gb, gob = OL.unpack(g), OL.unpack(go)
    for name, _ in OL.SHAPES:
        err = np.linalg.norm(gb[name] - gob[name])
        assert err <= 2.0 ** -8 * np.linalg.norm(gob[name]) + 1e-12, name
    # the padding columns of the output layer get exactly zero gradient
    assert np.all(gb["W3"][:, 3:] == 0) and np.all(gb["b3"][3:] == 0)


@pytest.mark.parametrize("rows,seed", [(64, 1), (96, 2), (2, 3), (2050, 4)])
def test_forward_and_backward_are_exact_on_exact_inputs(rows, seed):
    """Element by element: a wrong index, transpose, mask or bias sum in any
    of the six gradient blocks changes at least one value."""
    from tests.learn_exact import exact_case
    theta, fbits, T = exact_case(rows, seed)
    net = L.Net(theta, device=DEV)
    xb = torch.tensor(fbits.view(np.int16), device=DEV)
    y = net.forward(xb).cpu().numpy().astype(np.float64)
    X = OL.bf16_value(fbits)
    yo, _ = OL.forward(theta.astype(np.float64), X, emulate=True)
    np.testing.assert_array_equal(y, yo)
    loss = net.loss_grad(xb, torch.tensor(T, device=DEV))
    g = net.grad.cpu().numpy().astype(np.float64)
    lo, go = OL.loss_grad(theta.astype(np.float64), X, T.astype(np.float64), emulate=True)
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=1e-6)
    gb, gob = OL.unpack(g), OL.unpack(go)
    for name, _ in OL.SHAPES:
        np.testing.assert_array_equal(gb[name], gob[name], err_msg=name)


def test_adam_matches_the_oracle():
    rng = np.random.default_rng(7)
    theta = rng.normal(size=L.param_count()).astype(np.float32)
    net = L.Net(theta, device=DEV)
    th, m, v = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in range(1, 4):
        g = rng.normal(scale=10.0 ** -step, size=theta.size).astype(np.float32)
        net.grad.copy_(torch.tensor(g, device=DEV))
        net.adam_step(1e-3)
        th, m, v = OL.adam(th, g.astype(np.float64), m, v, step, 1e-3)
    got = net.theta.cpu().numpy()
    np.testing.assert_allclose(got, th, rtol=0, atol=4e-7 * np.abs(th).max() + 1e-8)
    np.testing.assert_array_equal(net.theta_bf16.cpu().numpy().view(np.uint16), OL.bf16_bits(got))


def test_gather_delta_displace_select_are_exact():
    rng = np.random.default_rng(8)
    src = torch.tensor(rng.integers(-30000, 30000, size=(500, 128)).astype(np.int16), device=DEV)
    idx = rng.integers(0, 500, size=333).astype(np.int32)
    out = torch.empty((333, 128), dtype=torch.int16, device=DEV)
    L.gather_rows(src, torch.tensor(idx, device=DEV), out)
    np.testing.assert_array_equal(out.cpu().numpy(), src.cpu().numpy()[idx])
    systems = [chain_system(40, 1), chain_system(25, 2), chain_system(50, 3)]
    sa = L.SystemArrays(systems, DEV)
    x0 = rng.normal(size=(sa.n, 3))
    x1 = x0 + rng.normal(scale=0.1, size=(sa.n, 3))
    t0, t1 = torch.tensor(x0, device=DEV), torch.tensor(x1, device=DEV)
    np.testing.assert_array_equal(L.delta(t0, t1).cpu().numpy(), (x1 - x0).astype(np.float32))
    disp = rng.normal(size=(sa.n, 16)).astype(np.float32)
    xd = L.displace(t0, torch.tensor(disp, device=DEV), 0.5).cpu().numpy()
    np.testing.assert_array_equal(xd, x0 + 0.5 * disp[:, :3].astype(np.float64))
    e_old = torch.tensor([1.0, 5.0, 2.0], dtype=torch.float64, device=DEV)
    e_new = torch.tensor([0.5, float("nan"), 2.0], dtype=torch.float64, device=DEV)
    xs, chosen, es = L.select(sa, t0, t1, e_old, e_new)
    assert chosen.cpu().tolist() == [1, 0, 0]
    assert es.cpu().tolist() == [0.5, 5.0, 2.0]
    want = x0.copy()
    want[:40] = x1[:40]
    np.testing.assert_array_equal(xs.cpu().numpy(), want)


def test_training_on_minimizer_pairs_generalizes_and_the_race_keeps_the_best():
    """End to end at a small scale: (start, minimum) pairs from the batched
    minimizer, training by the library's own kernels, then held-out chains.
    What the network gains over no displacement is its loss on held-out
    chains against the zero prediction's (the extended chains collapse
    towards their centroid, which the centroid-offset features expose).
    The learned start is the lowest-energy result of the race, and L-BFGS
    from it ends like a plain run, certified where it claims convergence."""
    import paper_1810_03358_amd as ff
    rng = np.random.default_rng(11)
    sizes = rng.integers(300, 600, size=56)
    systems = [chain_system(int(n), 500_000 + i) for i, n in enumerate(sizes)]
    train, val = systems[:48], systems[48:]
    data, res = L.make_pairs(train, lambda ss: ff.Context(ss), tol=1e-3, max_iter=20000, precision="fp32")
    data.finish()
    vdata, _ = L.make_pairs(val, lambda ss: ff.Context(ss), tol=1e-3, max_iter=20000, precision="fp32")
    vdata.finish()
    net = L.Net(seed=1, device=DEV)
    losses = L.train(net, data, epochs=40, batch=2048, lr=2e-3, lr_final=2e-5)
    assert losses[-1] < losses[0]
    zero = float(vdata.T.double().pow(2).mean().cpu())
    vloss = L.validation_loss(net, vdata)
    print(f"held-out loss {vloss:.4f} vs zero displacement {zero:.4f} (R2 {1 - vloss / zero:.3f})")
    assert vloss < 0.8 * zero
    rows = L.evaluate(net, val[:3], lambda s: ff.Context(s), max_iter=30000, control=False)
    for r in rows:
        print(r)
        ends = ("converged", "ls_failed", "max_iter")
        assert r["plain_term"] in ends and r["learned_term"] in ends
        if r["learned_term"] == "converged":
            assert r["learned_grad_inf"] < 1e-3
    # the race returns the candidate with the lowest energy after its probe
    s = val[3]
    sa = L.SystemArrays([s], DEV)
    pctx = ff.Context([s] * 3)
    x0 = torch.tensor(s["x"], dtype=torch.float64, device=DEV).contiguous()
    xw, best, pres = L.probe_start(pctx, sa, net, x0, (0.5, 1.0), probe_iters=100)
    energies = [r["energy"] for r in pres]
    assert best == int(np.argmin(energies))
    ctx = ff.Context(s)
    e = ctx.energy_grad(xw.contiguous(), "fp64", want_grad=False)[0].item()
    assert e == pytest.approx(energies[best], rel=1e-9)
