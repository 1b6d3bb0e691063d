"""Learned warm start (not in the paper): Python binding of include/ff_learn.h.

A small per-atom network predicts, from the 16 nearest neighbours of each
atom at the start point, the displacement that L-BFGS would apply to it on
the way to a local minimum.  The displaced start is kept only for systems
whose energy it lowers; L-BFGS then runs as usual and decides the result.
Every numerical step runs in the library's kernels; this module marshals
arguments, owns the device buffers (torch tensors) and drives training.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _native as N

NEIGHBORS, FEATURES, HIDDEN, OUT_PAD = N.FF_LEARN_NEIGHBORS, N.FF_LEARN_FEATURES, N.FF_LEARN_HIDDEN, N.FF_LEARN_OUT_PAD


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(status: int, where: str):
    if status != 0:
        raise RuntimeError(f"{where} failed ({status}): {N.learn_last_error()}")


def param_count() -> int:
    return int(N.load().ff_learn_param_count())


def init_params(seed: int = 0, out_scale: float = 1e-2) -> np.ndarray:
    """Packed FP32 parameters: He-normal hidden layers, an output layer scaled
    by out_scale (the first predictions are near zero), zero biases."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(scale=math.sqrt(2.0 / FEATURES), size=FEATURES * HIDDEN), np.zeros(HIDDEN),
             rng.normal(scale=math.sqrt(2.0 / HIDDEN), size=HIDDEN * HIDDEN), np.zeros(HIDDEN),
             rng.normal(scale=out_scale / math.sqrt(HIDDEN), size=HIDDEN * OUT_PAD), np.zeros(OUT_PAD)]
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == param_count()
    return theta


class SystemArrays:
    """Per-atom parameters and system map of a list of systems on the device
    (the feature kernel's inputs besides coordinates)."""

    def __init__(self, systems, device="cuda"):
        systems = list(systems)
        dev = torch.device(device)
        self.sizes = [int(s["n_atoms"]) for s in systems]
        self.n = sum(self.sizes)
        self.n_sys = len(systems)
        cat = lambda k: torch.tensor(np.concatenate([np.asarray(s[k], dtype=np.float64) for s in systems]),
                                     dtype=torch.float64, device=dev)
        self.q, self.sigma, self.eps = cat("q"), cat("sigma"), cat("eps")
        first = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int32)
        self.sys_first_host = first
        self.sys_first = torch.tensor(first, dtype=torch.int32, device=dev)
        self.atom_sys = torch.tensor(np.repeat(np.arange(self.n_sys, dtype=np.int32), self.sizes),
                                     dtype=torch.int32, device=dev)


def features(sa: SystemArrays, x: torch.Tensor, want_neighbors: bool = False, stream=None):
    """BF16 feature rows [n][FEATURES] (torch.int16 bit patterns) at x (FP64
    [n][3] device), and the neighbour lists if asked for."""
    if not (x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.numel() == 3 * sa.n):
        raise ValueError("x must be a contiguous float64 CUDA tensor with 3*n_atoms elements")
    f = torch.empty((sa.n, FEATURES), dtype=torch.int16, device=x.device)
    nb = torch.empty((sa.n, NEIGHBORS), dtype=torch.int32, device=x.device) if want_neighbors else None
    _check(N.load().ff_learn_features(sa.n_sys, sa.n, _ptr(x), _ptr(sa.q), _ptr(sa.sigma), _ptr(sa.eps),
                                      _ptr(sa.sys_first), _ptr(sa.atom_sys), _ptr(f), _ptr(nb), _stream_ptr(stream)),
           "ff_learn_features")
    return (f, nb) if want_neighbors else f


def gemm(a: torch.Tensor, sa, b: torch.Tensor, sb, m: int, n: int, k: int, bias=None, relu=False,
         out=None, out_bf16=None, stream=None):
    """Strided BF16 product through ff_learn_gemm (see the header)."""
    ldc = out.stride(0) if out is not None else 0
    ldcb = out_bf16.stride(0) if out_bf16 is not None else 0
    _check(N.load().ff_learn_gemm(m, n, k, _ptr(a), sa[0], sa[1], _ptr(b), sb[0], sb[1], _ptr(bias),
                                  1 if relu else 0, _ptr(out), ldc, _ptr(out_bf16), ldcb, _stream_ptr(stream)),
           "ff_learn_gemm")


def to_bf16(x: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(N.load().ff_learn_to_bf16(_ptr(x), x.numel(), _ptr(out), _stream_ptr(stream)), "ff_learn_to_bf16")
    return out


class Net:
    """The network's FP32 parameters, their BF16 copy and Adam state, on one
    device."""

    def __init__(self, theta=None, seed: int = 0, device="cuda"):
        self.device = torch.device(device)
        theta = init_params(seed) if theta is None else np.asarray(theta, dtype=np.float32)
        if theta.size != param_count():
            raise ValueError(f"expected {param_count()} parameters, got {theta.size}")
        self.theta = torch.tensor(theta, dtype=torch.float32, device=self.device)
        self.theta_bf16 = to_bf16(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.step = 0
        self._ws = None

    def _workspace(self, rows: int, backward: bool) -> tuple[torch.Tensor, int, int]:
        need = int(N.load().ff_learn_workspace_bytes(rows))
        if self._ws is None or self._ws.numel() < need + 256:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        return self._ws, (base + 255) // 256 * 256, need

    def forward(self, feats: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Network output [rows][OUT_PAD] (FP32) at BF16 features."""
        rows = feats.shape[0]
        out = out if out is not None else torch.empty((rows, OUT_PAD), dtype=torch.float32, device=self.device)
        _, ptr, need = self._workspace(rows, False)
        _check(N.load().ff_learn_forward(_ptr(self.theta), _ptr(self.theta_bf16), _ptr(feats), rows,
                                         C.c_void_p(ptr), need, _ptr(out), _stream_ptr(stream)), "ff_learn_forward")
        return out

    def loss_grad(self, feats: torch.Tensor, target: torch.Tensor, loss: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
        """Minibatch loss (device scalar, FP32); the gradient lands in self.grad."""
        rows = feats.shape[0]
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=self.device)
        _, ptr, need = self._workspace(rows, True)
        _check(N.load().ff_learn_backward(_ptr(self.theta), _ptr(self.theta_bf16), _ptr(feats), rows,
                                          C.c_void_p(ptr), need, _ptr(target), _ptr(self.grad), _ptr(loss),
                                          _stream_ptr(stream)), "ff_learn_backward")
        return loss

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        self.step += 1
        _check(N.load().ff_learn_adam(_ptr(self.theta), _ptr(self.theta_bf16), _ptr(self.grad), _ptr(self.m),
                                      _ptr(self.v), self.step, lr, beta1, beta2, eps, _stream_ptr(stream)),
               "ff_learn_adam")

    def params(self) -> np.ndarray:
        return self.theta.cpu().numpy()

    def save(self, path: str):
        np.savez(path, theta=self.params())

    @classmethod
    def load(cls, path: str, device="cuda") -> "Net":
        with np.load(path, allow_pickle=False) as z:
            return cls(z["theta"], device=device)


def gather_rows(src: torch.Tensor, idx: torch.Tensor, out: torch.Tensor, stream=None):
    rows = idx.numel()
    row_bytes = src.stride(0) * src.element_size()
    _check(N.load().ff_learn_gather_rows(_ptr(src), _ptr(idx), rows, row_bytes, _ptr(out), _stream_ptr(stream)),
           "ff_learn_gather_rows")


def delta(x_start: torch.Tensor, x_min: torch.Tensor, stream=None) -> torch.Tensor:
    """FP32 targets x_min - x_start [n][3]."""
    n = x_start.numel() // 3
    out = torch.empty((n, 3), dtype=torch.float32, device=x_start.device)
    _check(N.load().ff_learn_delta(_ptr(x_start), _ptr(x_min), n, _ptr(out), _stream_ptr(stream)), "ff_learn_delta")
    return out


def displace(x: torch.Tensor, disp: torch.Tensor, scale: float = 1.0, out=None, stream=None) -> torch.Tensor:
    n = x.numel() // 3
    out = out if out is not None else torch.empty_like(x)
    _check(N.load().ff_learn_displace(_ptr(x), _ptr(disp), n, float(scale), _ptr(out), _stream_ptr(stream)),
           "ff_learn_displace")
    return out


def select(sa: SystemArrays, x_old, x_new, e_old, e_new, out=None, e_out=None, stream=None):
    """(points, chosen[n_sys] int32, energies): per system the lower-energy
    point of x_old / x_new (x_new only if its energy is finite and lower).
    out / e_out may alias x_old / e_old."""
    out = out if out is not None else torch.empty_like(x_old)
    e_out = e_out if e_out is not None else torch.empty_like(e_old)
    chosen = torch.empty(sa.n_sys, dtype=torch.int32, device=x_old.device)
    _check(N.load().ff_learn_select(sa.n_sys, sa.n, _ptr(x_old), _ptr(x_new), _ptr(e_old), _ptr(e_new),
                                    _ptr(sa.atom_sys), _ptr(out), _ptr(chosen), _ptr(e_out), _stream_ptr(stream)),
           "ff_learn_select")
    return out, chosen, e_out


def warm_start(ctx, sa: SystemArrays, net: Net, x: torch.Tensor, scales=(0.25, 0.5, 1.0), precision="fp64",
               stream=None):
    """Learned start point(s): x + s * network(features(x)) for each s in
    `scales`, keeping per system the lowest energy among x and the candidates
    (evaluated by ctx in `precision`).  Returns (x_ws, scale index + 1 taken
    per system (0: x kept), energies at x_ws)."""
    f = features(sa, x, stream=stream)
    y = net.forward(f, stream=stream)
    best = x.clone()
    e_best, _ = ctx.energy_grad(x, precision, want_grad=False, stream=stream)
    taken = torch.zeros(sa.n_sys, dtype=torch.int32, device=x.device)
    for k, sc in enumerate(scales):
        cand = displace(x, y, sc, stream=stream)
        e_c, _ = ctx.energy_grad(cand, precision, want_grad=False, stream=stream)
        _, chosen, _ = select(sa, best, cand, e_best, e_c, out=best, e_out=e_best, stream=stream)
        taken = torch.where(chosen.bool(), k + 1, taken)
    return best, taken, e_best


class Dataset:
    """Training rows on the device: BF16 features at start points and FP32
    displacement targets (minimum - start)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.feats: list[torch.Tensor] = []
        self.targets: list[torch.Tensor] = []

    def add(self, feats: torch.Tensor, targets: torch.Tensor):
        self.feats.append(feats)
        self.targets.append(targets)

    def finish(self):
        self.X = torch.cat(self.feats) if len(self.feats) > 1 else self.feats[0]
        self.T = torch.cat(self.targets) if len(self.targets) > 1 else self.targets[0]
        self.feats, self.targets = [self.X], [self.T]
        return self

    @property
    def rows(self) -> int:
        return int(self.X.shape[0])


def make_pairs(systems, ctx_factory, tol: float = 1e-3, max_iter: int = 3000, precision="fp32", dataset=None,
               device="cuda"):
    """Minimize `systems` together (one batch context from ctx_factory) from
    their stored starts and add (features at start, minimum - start) rows to
    `dataset`.  Returns (dataset, per-system results)."""
    dataset = dataset if dataset is not None else Dataset(device)
    ctx = ctx_factory(systems)
    sa = SystemArrays(systems, device)
    x0 = torch.tensor(np.concatenate([s["x"] for s in systems]), dtype=torch.float64, device=device).contiguous()
    f = features(sa, x0)
    x = x0.clone()
    res = ctx.minimize(x, "lbfgs", tol=tol, max_iter=max_iter, precision=precision)
    dataset.add(f, delta(x0, x))
    ctx.close()
    return dataset, res


def train(net: Net, data: Dataset, epochs: int = 10, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          lr_final: float | None = None, log=None) -> list[float]:
    """Adam over shuffled minibatches (cosine decay from lr to lr_final).
    Returns the mean loss of each epoch."""
    rows = data.rows
    batch = min(batch, rows)
    steps_per_epoch = rows // batch
    fx = torch.empty((batch, FEATURES), dtype=torch.int16, device=net.device)
    tx = torch.empty((batch, 3), dtype=torch.float32, device=net.device)
    losses = torch.empty(max(steps_per_epoch, 1), dtype=torch.float32, device=net.device)
    rng = np.random.default_rng(seed)
    total = epochs * steps_per_epoch
    lr_final = lr if lr_final is None else lr_final
    out = []
    k = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(rows)[: steps_per_epoch * batch].astype(np.int32), device=net.device)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            gather_rows(data.X, idx, fx)
            gather_rows(data.T, idx, tx)
            net.loss_grad(fx, tx, losses[s:s + 1])
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / max(total, 1)))
            net.adam_step(cur)
            k += 1
        out.append(float(losses[:steps_per_epoch].double().mean().cpu()))
        if log:
            log(f"epoch {ep}: loss {out[-1]:.5f}")
    return out


def validation_loss(net: Net, data: Dataset, chunk: int = 65536) -> float:
    """Mean loss over every row of `data` (the gradient buffer is reused)."""
    loss = torch.empty(1, dtype=torch.float32, device=net.device)
    total = 0.0
    for r0 in range(0, data.rows, chunk):
        r1 = min(r0 + chunk, data.rows)
        net.loss_grad(data.X[r0:r1], data.T[r0:r1], loss)
        total += float(loss.cpu()[0]) * (r1 - r0)
    return total / data.rows


def _sync_time(fn):
    torch.cuda.synchronize()
    t = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t[0].record()
    out = fn()
    t[1].record()
    torch.cuda.synchronize()
    return out, t[0].elapsed_time(t[1]) / 1e3


def probe_start(probe_ctx, sa: SystemArrays, net: Net, x: torch.Tensor, scales=(0.5, 1.0), probe_iters: int = 200,
                tol: float = 1e-3, precision="fp32", transform=None, stream=None):
    """Learned start of one system, chosen by a short race: x and
    x + s * network(features(x)) for each s in `scales` are minimized side by
    side (probe_ctx: a batch context holding
    1 + len(scales) copies of the system) for probe_iters L-BFGS iterations,
    and the lowest-energy result is returned as (point [n][3], index of the
    winner (0: x itself), per-candidate results).  The start energy is no
    guide here: a displaced start that brings the atoms most of the way to
    the minimum usually has a new clash, so its energy is higher until the
    first iterations have relieved it.  `transform(y)`, if given, replaces
    the network's output before it is applied (the evaluation's controls)."""
    n3 = x.numel()
    k = 1 + len(scales)
    if probe_ctx.n_sys != k or probe_ctx.n * 3 != k * n3:
        raise ValueError("probe context must hold 1 + len(scales) copies of the system")
    f = features(sa, x, stream=stream)
    y = net.forward(f, stream=stream)
    if transform is not None:
        y = transform(y)
    xb = torch.empty(k * n3, dtype=torch.float64, device=x.device)
    xb[:n3].copy_(x.reshape(-1))
    for i, sc in enumerate(scales):
        displace(x, y, sc, out=xb[(i + 1) * n3:(i + 2) * n3], stream=stream)
    res = probe_ctx.minimize(xb, "lbfgs", tol=tol, max_iter=probe_iters, precision=precision, stream=stream)
    e = [r["energy"] if math.isfinite(r["energy"]) else math.inf for r in res]
    best = int(np.argmin(e))
    return xb[best * n3:(best + 1) * n3].reshape(-1, 3), best, res


def random_directions(seed: int):
    """A control for the evaluation: the network's per-atom displacement
    lengths in uniformly random directions (seeded torch generator)."""
    def transform(y: torch.Tensor) -> torch.Tensor:
        g = torch.Generator(device=y.device)
        g.manual_seed(seed)
        r = torch.randn((y.shape[0], 3), generator=g, device=y.device, dtype=torch.float32)
        r = r / r.norm(dim=1, keepdim=True) * y[:, :3].norm(dim=1, keepdim=True)
        out = torch.zeros_like(y)
        out[:, :3] = r
        return out
    return transform


def race_length(n_atoms: int) -> int:
    """Iterations of the race for a system of n_atoms: a displaced start
    needs longer to relieve its clashes in a larger system (measured: 200
    suffice at 2,000 atoms, 1,000 are needed at 10,000)."""
    return min(1000, max(200, n_atoms // 10))


def evaluate(net: Net, systems, ctx_factory, tol: float = 1e-3, max_iter: int = 60000, precision="fp32",
             scales=(0.5, 1.0), probe_iters: int | None = None, control: bool = True, random_control: bool = False,
             device="cuda", log=None) -> list[dict]:
    """Time to |grad E|_inf < tol of each system alone: plain L-BFGS from its
    stored start, and the learned start (probe_start) followed by L-BFGS
    from the winner, with features, network, the race and the final run all
    inside the timed region.  With `control`, also L-BFGS restarted after
    probe_iters iterations from the stored start alone (what the race does
    without the network); with `random_control`, the same race with the
    network's displacement lengths in random directions.  Contexts are built outside the timed regions;
    each time is bracketed by device synchronisations.  probe_iters=None
    takes race_length(n_atoms) per system."""
    rows = []
    fixed_probe = probe_iters
    for i, s in enumerate(systems):
        probe_iters = fixed_probe if fixed_probe is not None else race_length(int(s["n_atoms"]))
        ctx = ctx_factory(s)
        pctx = ctx_factory([s] * (1 + len(scales)))
        sa = SystemArrays([s], device)
        x0 = torch.tensor(s["x"], dtype=torch.float64, device=device).contiguous()
        xp = x0.clone()
        rp, tp = _sync_time(lambda: ctx.minimize(xp, "lbfgs", tol=tol, max_iter=max_iter, precision=precision))

        def raced(transform=None):
            xw, best, pres = probe_start(pctx, sa, net, x0, scales, probe_iters, tol, precision, transform)
            xw = xw.contiguous()
            if pres[best]["term"] == 0:
                return pres[best], best, pres, 0
            r = ctx.minimize(xw, "lbfgs", tol=tol, max_iter=max_iter - probe_iters, precision=precision)
            return r, best, pres, r["iters"]
        (rl, best, pres, more), tl = _sync_time(raced)
        if random_control:
            (rr, best_r, pres_r, more_r), tr = _sync_time(lambda: raced(random_directions(1000 + i)))
        if control:
            xc = x0.clone()

            def restarted():
                r1 = ctx.minimize(xc, "lbfgs", tol=tol, max_iter=probe_iters, precision=precision)
                if r1["term"] == 0:
                    return r1, r1["iters"]
                r2 = ctx.minimize(xc, "lbfgs", tol=tol, max_iter=max_iter - probe_iters, precision=precision)
                return r2, r1["iters"] + r2["iters"]
            (rc, itc), tc = _sync_time(restarted)
        row = dict(n=int(s["n_atoms"]), plain_time=tp, plain_iters=rp["iters"], plain_evals=rp["evals"],
                   plain_term=rp["term_name"], plain_energy=rp["energy"], plain_grad_inf=rp["grad_inf"],
                   learned_time=tl, learned_iters=pres[best]["iters"] + more,
                   learned_evals=sum(r["evals"] for r in pres) + (rl["evals"] if more else 0),
                   learned_term=rl["term_name"], learned_energy=rl["energy"], learned_grad_inf=rl["grad_inf"],
                   scale_taken=(0.0 if best == 0 else float(scales[best - 1])), race_iters=probe_iters,
                   probe_energies=[r["energy"] for r in pres])
        if control:
            row.update(control_time=tc, control_iters=itc, control_term=rc["term_name"], control_energy=rc["energy"])
        if random_control:
            row.update(random_time=tr, random_iters=pres_r[best_r]["iters"] + more_r, random_term=rr["term_name"],
                       random_energy=rr["energy"], random_winner=best_r)
        rows.append(row)
        if log:
            log(f"system {i} ({row['n']} atoms): plain {tp:.2f} s {rp['iters']} it {rp['term_name']} "
                f"E {rp['energy']:.6e} | learned {tl:.2f} s {row['learned_iters']} it {rl['term_name']} "
                f"E {rl['energy']:.6e} scale {row['scale_taken']}"
                + (f" | restart {tc:.2f} s {itc} it {rc['term_name']} E {rc['energy']:.6e}" if control else "")
                + (f" | random {tr:.2f} s {rr['term_name']} E {rr['energy']:.6e} winner {best_r}"
                   if random_control else ""))
        ctx.close()
        pctx.close()
    return rows
