"""CPU checks of the C ABI: the library loads, exports every declared entry
point, sizes workspaces and rejects bad input on the host (no GPU calls)."""
import ctypes as C
import os
import re

import pytest

import paper_1810_03358_amd as ff
from paper_1810_03358_amd import _native as N
from synth import chain_system
from tests.systems import make_system

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions(header=None):
    names = [header] if header else sorted(f for f in os.listdir(INCLUDE) if f.endswith(".h"))
    found = set()
    for h in names:
        text = open(os.path.join(INCLUDE, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        found |= set(re.findall(r"\b(ff_[a-z0-9_]+)\s*\(", text))
    return sorted(found)


def test_header_and_binding_agree():
    assert declared_functions("ff.h") == sorted(N.EXPORTS)
    assert declared_functions("ff_learn.h") == sorted(N.LEARN_EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = N.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_default_params():
    p = N.FFMinParams()
    N.load().ff_default_params(C.byref(p))
    assert (p.method, p.m, p.tol, p.max_iter, p.precision, p.linesearch, p.ls_K) == (
        ff.FF_LBFGS, 10, 1e-3, 2000, ff.FF_FP64, ff.FF_LS_DEFAULT, 2)
    assert (p.h_init, p.k_plus, p.k_minus, p.eps_h, p.cg_restart, p.flags) == (0.1, 2.0, 0.5, 1e-10, 0, 0)
    assert (p.cg_beta, p.ls_par_g0, p.fgm_restart) == (ff.FF_CG_PRP, 1, 0)
    assert (p.hb_alpha, p.hb_beta) == (0.0, 0.0)


@pytest.mark.parametrize("n", [1, 2, 63, 512, 513, 10_000, 50_000])
def test_workspace_bytes_grows_with_size(n):
    s = make_system(np_zeros(n))
    b0 = ff.workspace_bytes(s, 0)
    assert b0 > 0 and b0 % 256 == 0
    # the vectors are sized for the largest memory; only the accept pass's
    # reduction rows (1 + m) grow with m
    b10 = ff.workspace_bytes(s, 10)
    assert b0 <= b10 <= b0 + 64 * 11 * 6 * 8 + 256


def np_zeros(n):
    import numpy as np
    return np.zeros((n, 3))


def test_workspace_bytes_rejects_bad_sizes():
    s = make_system(np_zeros(4))
    assert ff.workspace_bytes(s, 33) == 0
    assert ff.workspace_bytes(s, -1) == 0


def _create_status(system, m_max=10, ws_ptr=256, ws_bytes=1 << 40):
    hs = ff.HostSystem(system)
    ctx = C.c_void_p()
    return N.load().ff_create(C.byref(hs.c), C.c_void_p(ws_ptr), ws_bytes, m_max, None, C.byref(ctx))


def test_create_rejects_bad_input_before_touching_the_device():
    good = chain_system(20, 1)
    bad_bond = dict(good, bonds=good["bonds"].copy())
    bad_bond["bonds"][3, 1] = 20
    assert _create_status(bad_bond) == ff.FF_ERR_ARG
    assert "out of range" in N.last_error()
    neg = dict(good, sigma=-good["sigma"])
    assert _create_status(neg) == ff.FF_ERR_ARG
    assert _create_status(good, ws_ptr=257) == ff.FF_ERR_WORKSPACE
    assert _create_status(good, ws_bytes=1024) == ff.FF_ERR_WORKSPACE
    assert _create_status(good, m_max=40) == ff.FF_ERR_ARG
    self_bond = dict(good, bonds=good["bonds"].copy())
    self_bond["bonds"][2] = (5, 5)
    assert _create_status(self_bond) == ff.FF_ERR_ARG


def test_product_package_does_not_import_the_oracle():
    import ast
    pkg = os.path.dirname(ff.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(root, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, (ast.Import, ast.ImportFrom)):
                        names = [a.name for a in node.names] + [getattr(node, "module", "") or ""]
                        assert not any(n.split(".")[0] == "oracle" for n in names), f


def test_batch_workspace_and_validation():
    import numpy as np
    a, b = chain_system(50, 1), chain_system(300, 2)
    hs = [ff.HostSystem(a), ff.HostSystem(b)]
    arr = (N.FFSystem * 2)(*[h.c for h in hs])
    lib = N.load()
    nb = lib.ff_workspace_bytes_batch(arr, 2, 10)
    assert nb > 0 and nb % 256 == 0
    assert lib.ff_workspace_bytes_batch(arr, 0, 10) == 0
    bad = dict(b, bonds=b["bonds"].copy())
    bad["bonds"][7, 0] = 300
    hs2 = [ff.HostSystem(a), ff.HostSystem(bad)]
    arr2 = (N.FFSystem * 2)(*[h.c for h in hs2])
    ctx = C.c_void_p()
    st = lib.ff_create_batch(arr2, 2, C.c_void_p(256), 1 << 40, 10, None, C.byref(ctx))
    assert st == ff.FF_ERR_ARG and "system 1" in N.last_error()


def test_tile_configs_and_tiled_workspace():
    cfgs = ff.tile_configs()
    assert len(cfgs) >= 4
    for block, w32, i32, w64, i64 in cfgs:
        assert block == 64 * w32 * i32 == 64 * w64 * i64
    lib = N.load()
    s = chain_system(700, 3)
    arr = (N.FFSystem * 1)(ff.HostSystem(s).c)
    for k in range(len(cfgs)):
        for chunk in (1, 4, 16):
            b = lib.ff_workspace_bytes_tiled(arr, 1, 10, k, chunk, 0)
            assert b > 0 and b % 256 == 0
            # separate FP64 chunk length: its own chunk table, partial rows sized for the longer table
            assert lib.ff_workspace_bytes_tiled(arr, 1, 10, k, chunk, 1) >= b
    assert lib.ff_workspace_bytes_tiled(arr, 1, 10, len(cfgs), 4, 0) == 0
    assert lib.ff_workspace_bytes_tiled(arr, 1, 10, 0, 0, 0) == 0
    assert lib.ff_workspace_bytes_tiled(arr, 1, 10, 0, 5000, 0) == 0
    assert lib.ff_workspace_bytes_tiled(arr, 1, 10, 0, 4, 5000) == 0
    assert lib.ff_workspace_bytes_tiled(arr, 1, 10, 0, 4, -1) == 0
    need = lib.ff_autotune_workspace_bytes(arr, 1)
    assert need >= max(lib.ff_workspace_bytes_tiled(arr, 1, 0, k, c, 0) for k in range(len(cfgs)) for c in (1, 16))
    assert lib.ff_tile_config_info(len(cfgs), None, None, None, None, None) == ff.FF_ERR_ARG


def test_create_tiled_rejects_bad_tiling_before_touching_the_device():
    lib = N.load()
    s = chain_system(100, 3)
    arr = (N.FFSystem * 1)(ff.HostSystem(s).c)
    ctx = C.c_void_p()
    assert lib.ff_create_tiled(arr, 1, C.c_void_p(256), 1 << 40, 10, -1, 4, 0, None, C.byref(ctx)) == ff.FF_ERR_ARG
    assert lib.ff_create_tiled(arr, 1, C.c_void_p(256), 1 << 40, 10, 99, 4, 0, None, C.byref(ctx)) == ff.FF_ERR_ARG
    assert lib.ff_create_tiled(arr, 1, C.c_void_p(256), 1 << 40, 10, 0, 0, 0, None, C.byref(ctx)) == ff.FF_ERR_ARG
    assert lib.ff_create_tiled(arr, 1, C.c_void_p(256), 1 << 40, 10, 0, 4, 5000, None, C.byref(ctx)) == ff.FF_ERR_ARG
    assert lib.ff_create_tiled(arr, 1, C.c_void_p(256), 1024, 10, 0, 4, 0, None, C.byref(ctx)) == ff.FF_ERR_WORKSPACE


def test_energy_profile_rejects_bad_arguments_on_the_host():
    lib = N.load()
    t = (C.c_double * 2)(0.0, float("nan"))
    out = (C.c_double * 2)()
    ctx = C.c_void_p(0)
    assert lib.ff_energy_profile(ctx, C.c_void_p(256), t, 2, out, 0, None) == ff.FF_ERR_ARG


def test_far_exclusions_are_accepted_and_sized():
    """Bonds between atoms more than 64 apart (cross-links, ring closures) get
    per-unit exclusion masks: the workspace grows by one mask block per pair
    unit that holds such a pair."""
    from tests.systems import crosslinked_chain
    plain = chain_system(1100, 5)
    linked = crosslinked_chain(1100, 5)
    lib = N.load()
    a = (N.FFSystem * 1)(ff.HostSystem(plain).c)
    b = (N.FFSystem * 1)(ff.HostSystem(linked).c)
    for cfg, block in enumerate(t[0] for t in ff.tile_configs()):
        wa = lib.ff_workspace_bytes_tiled(a, 1, 10, cfg, 2, 0)
        wb = lib.ff_workspace_bytes_tiled(b, 1, 10, cfg, 2, 0)
        assert wa > 0 and wb > wa


def test_learn_entry_points_reject_bad_arguments_on_the_host():
    lib = N.load()
    assert lib.ff_learn_param_count() == 128 * 128 * 2 + 128 * 16 + 128 * 2 + 16
    assert lib.ff_learn_workspace_bytes(0) == 0
    assert lib.ff_learn_workspace_bytes(100) > 100 * 128 * 12
    nul = None
    p = C.c_void_p(256)
    assert lib.ff_learn_features(0, 10, p, p, p, p, p, p, p, nul, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_features(1, 10, p, nul, p, p, p, p, p, nul, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_gemm(0, 1, 1, p, 1, 1, p, 1, 1, nul, 0, p, 1, nul, 1, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_gemm(1, 1, 1, p, 1, 1, p, 1, 1, nul, 0, nul, 1, nul, 1, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_forward(p, p, p, 10, p, 16, p, nul) == ff.FF_ERR_WORKSPACE
    assert lib.ff_learn_forward(p, p, p, 10, C.c_void_p(257), 1 << 30, p, nul) == ff.FF_ERR_WORKSPACE
    ws1 = lib.ff_learn_workspace_bytes(10)
    assert lib.ff_learn_backward(p, p, p, 10, p, ws1 - 1024, p, p, p, nul) == ff.FF_ERR_WORKSPACE
    assert "workspace" in N.learn_last_error()
    assert lib.ff_learn_adam(p, nul, p, p, p, 0, 1e-3, 0.9, 0.999, 1e-8, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_adam(p, nul, p, p, p, 1, 0.0, 0.9, 0.999, 1e-8, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_gather_rows(p, p, 5, 6, p, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_displace(p, p, 5, float("inf"), p, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_select(1, 0, p, p, p, p, p, p, nul, nul, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_to_bf16(p, 0, p, nul) == ff.FF_ERR_ARG
    assert lib.ff_learn_delta(p, nul, 4, p, nul) == ff.FF_ERR_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(INCLUDE)
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_output_buffers_are_checked_before_any_kernel_writes_them():
    import torch
    from paper_1810_03358_amd import _out_tensor
    x = torch.zeros(30, dtype=torch.float64)      # stands in for checked coordinates
    with pytest.raises(ValueError, match="float64"):
        _out_tensor(torch.zeros(30, dtype=torch.float32), 30, x, "out_g")
    with pytest.raises(ValueError, match="elements"):
        _out_tensor(torch.zeros(0, dtype=torch.float64), 1, x, "out_e")
    with pytest.raises(ValueError, match="elements"):
        _out_tensor(torch.zeros(29, dtype=torch.float64), 30, x, "out_g")
    with pytest.raises(ValueError, match="contiguous"):
        _out_tensor(torch.zeros(60, dtype=torch.float64)[::2], 30, x, "out_g")
    with pytest.raises(ValueError, match="on meta"):
        _out_tensor(torch.zeros(30, dtype=torch.float64, device="meta"), 30, x, "out_g")
    t = torch.zeros(30, dtype=torch.float64)
    assert _out_tensor(t, 30, x, "out_g") is t


def _noalloc_status(system, precision=ff.FF_FP64):
    hs = ff.HostSystem(system)
    # any non-null pointers: every failure below is found before device work
    return N.load().ff_energy_grad_noalloc(C.byref(hs.c), C.c_void_p(256), C.c_void_p(512), None, precision, None)


def test_noalloc_rejects_oversized_and_bad_input_before_touching_the_device():
    big = make_system(np_zeros(40_000))
    assert _noalloc_status(big) == ff.FF_ERR_UNSUPPORTED
    assert "scratch" in N.last_error() and str(N.FF_NOALLOC_SCRATCH_BYTES) in N.last_error()
    good = chain_system(20, 1)
    bad = dict(good, bonds=good["bonds"].copy())
    bad["bonds"][3, 1] = 20
    assert _noalloc_status(bad) == ff.FF_ERR_ARG and "bond 3" in N.last_error()
    assert _noalloc_status(good, precision=7) == ff.FF_ERR_ARG
    hs = ff.HostSystem(good)
    assert N.load().ff_energy_grad_noalloc(C.byref(hs.c), None, C.c_void_p(512), None, 0, None) == ff.FF_ERR_ARG


def test_noalloc_scratch_limit_matches_the_header():
    text = open(os.path.join(INCLUDE, "ff.h")).read()
    m = re.search(r"#define FF_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == N.FF_NOALLOC_SCRATCH_BYTES


def test_bench_cpu_baseline_legs_on_a_small_chain():
    """The benchmark's oracle legs (no GPU): the all-threads rate, the
    one-thread row sample with the CPU model, and the timed oracle solve
    that --solve --oracle reports beside the GPU's."""
    import sys
    root = os.path.dirname(INCLUDE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import bench
    import oracle
    s = chain_system(120, 3)
    cb = bench.cpu_baseline(s, s["x"], seconds=0.2)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] == oracle.num_threads()
    assert cb["one_core"]["cores"] == 1 and cb["one_core"]["value"] > 0 and cb["cpu_model"]
    threads = oracle.num_threads()
    o = bench.oracle_solve(s, "lbfgs", 50, threads=1)
    assert oracle.num_threads() == threads          # restored
    assert o["cores"] == 1 and o["iters"] == 50 and o["term"] == "max_iter" and o["x"].shape == (360,)
    ref = oracle.minimize(lambda v: oracle.energy_grad(oracle.System(s), v.reshape(-1, 3)), s["x"].ravel(),
                          oracle.MinParams(method=oracle.LBFGS, m=10, tol=1e-3, max_iter=50))
    assert o["energy"] == ref.f and o["evals"] == ref.evals
