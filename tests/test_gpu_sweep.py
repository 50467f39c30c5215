"""End-to-end GPU parity of the TT-RBKI sweep against the float64 CPU oracle.

Both sides consume the same tensor and the same seeded Omega (each from its own
Philox4x64-10 implementation).  Compared quantities are unique regardless of the
gauge of the cores: the relative error eps = ||X - Xhat|| / ||X||, the relative
reconstruction difference delta_rec = ||Xhat_gpu - Xhat_oracle|| / ||X|| (entrywise on
the host) and, per bond, the sine of the largest principal angle between the left
interface subspaces (Definition 2).  Tolerances: float64 1e-10, float32 1e-5 on eps and
delta_rec; bfloat16 streaming must match the oracle's eps to 1% (the matched-error bar of
the precision comparison) where eps >= 5e-3, else stay within 2^-9 (its operand rounding)
of it; the cores must be left-orthonormal.

Principal angles follow a Wedin-style bound: a perturbation E of the unfolding moves its
leading r-dimensional subspace by sin(theta) <= ||E|| / gap, gap = sigma_r - sigma_{r+1}
(Ritz values of the Krylov space for regular modes, singular values for saturated ones),
and the interface at bond k inherits the moves of the bonds before it.  ||E|| is taken
as C * sigma_1 with C = 1e-10 (float64) and 1e-4 (float32), about 100 times the rounding
of the streamed products.
"""
import math

import numpy as np
import pytest
import torch

import paper_2308_01480_amd as ttr
import synth
from oracle import metrics, ttrbki
from tests.gpu_util import announce, dev_compare, dev_interface_sines, stored_f64, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}
ORTH = {"f64": 1e-12, "f32": 1e-12, "bf16": 1e-12}
WEDIN = {"f64": 1e-10, "f32": 1e-4}


def wedin_bounds(modes, c):
    """Per-bond bound on sin(theta) between two runs whose unfoldings differ by c * sigma_1."""
    out, acc = [], 0.0
    for mi in modes:
        if mi.kind != "identity" and mi.ritz is not None:
            sig = np.sqrt(np.maximum(np.asarray(mi.ritz, dtype=np.float64), 0.0))
            sig = np.concatenate([sig, np.zeros(max(0, mi.r + 1 - len(sig)))])  # fewer kept directions than r
            gap = sig[mi.r - 1] - sig[mi.r]
            acc += c * sig[0] / gap if gap > 0 else math.inf
        out.append(min(1.0, acc))
    return out


def run_pair(X, ranks, q, p, seed, dt, label, device_metrics=False, method="rbki", literal=False, krylov="auto"):
    """GPU sweep vs oracle on the same stored tensor.  With ``device_metrics`` the checker
    sums (eps, delta_rec, principal angles) run as plain torch float64 on the GPU instead of
    numpy on the host (same definitions; for tensors of 1e9 entries).  ``method`` and
    ``literal`` select TT-rSI / TT-rSVD and the printed truncation (oracle: tt_variant)."""
    announce(f"{label} {dt} dims={X.shape} ranks={ranks} q={q} p={p} method={method} literal={literal} "
             f"krylov={krylov}")
    x = to_dev(X, dt)
    Xs = stored_f64(x)  # the stored values (float32 / bf16 rounding included) are the input of both sides
    cores = ttr.tt_rbki(x, ranks, q, p, seed=seed, method=method, literal=literal, krylov=krylov)
    err = ttr.tt_error(x, cores).cpu().numpy()
    g = [c.cpu().numpy() for c in cores]
    announce(f"{label} {dt} oracle")
    if method == "rbki" and not literal:
        o, modes = ttrbki.tt_rbki(Xs, ranks, q, p, seed=seed, precision=dt, diagnostics=True,
                                  residuals=not device_metrics)
    else:
        o = ttrbki.tt_variant(Xs, ranks, q, p, seed=seed, method=method, truncation="first" if literal else "ritz",
                              precision=dt)
        modes = None
    if device_metrics:
        del Xs
        ea, eb, x2, dd = dev_compare(x, o, g)
        e_o, e_g = math.sqrt(ea / x2), math.sqrt(eb / x2)
        drec = math.sqrt(dd / x2)
        sines = dev_interface_sines(g, o)
    else:
        x2 = float(np.sum(Xs * Xs))
        e_o = metrics.rel_error(Xs, o)
        e_g = metrics.rel_error(Xs, g)
        drec = math.sqrt(metrics.rec_diff_sq(g, o) / x2) if x2 > 0 else math.sqrt(metrics.rec_diff_sq(g, o))
        sines = metrics.interface_sines(g, o)
    del x
    e_dev = math.sqrt(err[0] / err[1]) if err[1] > 0 else math.sqrt(err[0])
    print(f"[gpu-case]   eps_oracle={e_o:.10e} eps_gpu={e_g:.10e} dev_eps={e_dev:.10e} delta_rec={drec:.3e}",
          flush=True)
    if dt == "bf16":
        # bfloat16 streaming: the streamed operands carry 2^-9 relative rounding, which
        # perturbs the Krylov space at that level.  Where the residual dominates it
        # (eps >= 5e-3) the error must match the oracle's on the same stored input to 1%
        # (the matched-error bar); below, the rounding itself shows in eps and the error
        # must stay within 2^-9 of the oracle's.  delta_rec and the angles are reported.
        print(f"[gpu-case]   sin_theta={['%.2e' % v for v in sines]}", flush=True)
        assert abs(e_g - e_o) <= (1e-2 * e_o if e_o >= 5e-3 else 2.0 ** -9)
    else:
        bnd = wedin_bounds(modes, WEDIN[dt]) if modes is not None else [1.0] * len(sines)
        print(f"[gpu-case]   sin_theta={['%.2e' % v for v in sines]} bound={['%.2e' % v for v in bnd]}", flush=True)
        assert abs(e_g - e_o) <= TOL[dt]
        assert drec <= TOL[dt]
        for k, (sv, bv) in enumerate(zip(sines, bnd)):
            assert sv <= bv, (k + 1, sv, bv)
    assert abs(e_dev - e_g) <= 1e-12 + 1e-9 * e_g
    assert metrics.left_orthonormality(g) <= ORTH[dt]
    return g, o


CASES = [
    ("tt20x4", None, {}),
    ("tt48x5", (16, 16, 16, 16, 16), {}),
    ("tt24x6", (10, 10, 10, 10, 10, 10), {}),
    ("tt8x10", (6,) * 8, {}),
    ("odeco256x4", (64, 64, 64, 64), {"signal_rank": 24, "ranks": 12, "p": 4}),
    # the 256^4 run parameters (r = 32, p = 8, q = 4: w = 200) on a TT signal: a regular first
    # mode with a 200 x 200 Rayleigh-Ritz matrix and a regular second mode with m = 8192 rows
    # (two-pass Krylov products)
    ("odeco256x4", (256, 256, 64, 16), {"signal": "tt", "signal_rank": 40}),
]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name,dims,chg", CASES)
def test_workload_twins(name, dims, chg, dt):
    w = synth.workload(name)
    if dims:
        w = synth.scaled_down(w, dims, **chg)
    X = synth.build_host(w)
    run_pair(X, w.target_ranks(), w.q, w.p, w.omega_seed, dt, w.name)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name,dims,chg", [CASES[0], CASES[1], CASES[4], CASES[5]])
def test_workload_twins_streamed(name, dims, chg, dt):
    # the planner takes the Krylov products of short unfoldings (m <= 256) through A A^T;
    # the streamed A (A^T Z) kernels on the same modes, forced
    w = synth.workload(name)
    if dims:
        w = synth.scaled_down(w, dims, **chg)
    X = synth.build_host(w)
    pl = ttr.plan(list(X.shape), w.target_ranks(), w.q, w.p, torch.float32, krylov="streamed")
    assert not any(pl.gram_first[k] for k in range(pl.d - 1))
    run_pair(X, w.target_ranks(), w.q, w.p, w.omega_seed, dt, w.name, krylov="streamed")


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_edge_shapes(dt):
    rng = np.random.default_rng(5)
    # odd sizes: rows of odd length are not 16-byte aligned; m not a multiple of 16
    run_pair(rng.standard_normal((7, 9, 11, 13)), [3, 5, 4], 2, 2, 1, dt, "odd-sizes")
    # matrix case (d = 2), one regular mode with a ragged last tile
    run_pair(rng.standard_normal((40, 1001)), [6], 1, 3, 2, dt, "matrix")
    # a regular mode with m > 512 (two-pass Krylov kernels), q = 0 (sketch only)
    run_pair(rng.standard_normal((30, 30, 700)), [25, 10], 0, 5, 3, dt, "q0-two-pass")
    run_pair(rng.standard_normal((30, 30, 700)), [25, 10], 2, 5, 3, dt, "tall-two-pass")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_split_operand_products(dt):
    # mode 2 is a tall, wide float32 unfolding (1536 x 32768): in the float32 tier its
    # two-pass Krylov products and its carry run on the bf16 matrix cores with three-way
    # split operands, held to the float32 bars like every other float32 product
    X = synth.tt_full_host(synth.tt_cores_random((32, 48, 256, 128), 8, 1.0, 31))
    rng = np.random.default_rng(32)
    E = rng.standard_normal(X.shape)
    X = X + 1e-2 * np.linalg.norm(X) / np.linalg.norm(E) * E
    pl = ttr.plan(list(X.shape), [32, 24, 24], 2, 8, torch.float32)
    assert pl.kinds == ["identity", "regular", "regular"] and int(pl.m[1]) == 1536 and int(pl.n[1]) == 32768
    run_pair(X, [32, 24, 24], 2, 8, 5, dt, "split-operands")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_split_operand_products_ragged(dt):
    # the same path on a ragged mode (1440 x 33667): a partial last row chunk of the A^T Z
    # kernel, a partial last column tile, rows of odd length (no 16-byte loads of A) and
    # a W plane pitch padded past n
    dims = (32, 45, 257, 131)
    X = synth.tt_full_host(synth.tt_cores_random(dims, 8, 1.0, 41))
    rng = np.random.default_rng(42)
    E = rng.standard_normal(X.shape)
    X = X + 1e-2 * np.linalg.norm(X) / np.linalg.norm(E) * E
    pl = ttr.plan(list(dims), [32, 24, 24], 2, 8, torch.float32)
    assert int(pl.m[1]) == 1440 and int(pl.n[1]) == 33667 and int(pl.two_pass[1]) == 1
    run_pair(X, [32, 24, 24], 2, 8, 5, dt, "split-operands-ragged")


@pytest.mark.parametrize("dims,ranks,q,p", [
    # m_pad <= 128 (four row steps), r = 12 (one carry row block), next sketch width 16
    ((100, 40, 64, 32), [12, 10, 8], 2, 6),
    # m_pad 208 (eight row steps), r = 20, next sketch width 24 (padded to 32); 60 tiles per
    # block over 42 work-groups, so the last groups of each block take no tile
    ((200, 24, 96, 40), [20, 16, 10], 2, 8),
])
def test_carry_with_next_sketch(dims, ranks, q, p):
    # bfloat16 mode 1 is a short unfolding with a float32 carry and mode 2 a regular
    # two-pass mode: the carry pass also forms mode 2's sketch (its Omega drawn transposed,
    # products on the float32 matrix cores from the carry accumulators)
    X = synth.tt_full_host(synth.tt_cores_random(dims, 8, 1.0, 51))
    rng = np.random.default_rng(52)
    E = rng.standard_normal(X.shape)
    X = X + 1e-2 * np.linalg.norm(X) / np.linalg.norm(E) * E
    pl = ttr.plan(list(dims), ranks, q, p, torch.bfloat16)
    assert pl.kinds[0] == "regular" and pl.kinds[1] == "regular" and not pl.gram_first[1]
    run_pair(X, ranks, q, p, 7, "bf16", "carry-next-sketch")


def test_exact_low_rank_and_zero():
    X = synth.tt_full_host(synth.tt_cores_random((9, 10, 11, 12), 3, 1.0, 77))
    g, _ = run_pair(X, [5, 5, 5], 2, 3, 0, "f64", "exact-rank3")
    assert metrics.rel_error(X, g) <= 1e-12
    Z = np.zeros((6, 7, 8))
    x = to_dev(Z, "f64")
    cores = ttr.tt_rbki(x, [3, 3], 1, 2, seed=0)
    g = [c.cpu().numpy() for c in cores]
    assert metrics.left_orthonormality(g) <= 1e-14
    assert metrics.errors(Z, g)[0] == 0.0


def test_deterministic():
    w = synth.scaled_down(synth.workload("tt48x5"), (16, 16, 16, 16, 16))
    x = to_dev(synth.build_host(w), "f32")
    a = ttr.tt_rbki(x, w.target_ranks(), w.q, w.p, seed=0)
    b = ttr.tt_rbki(x, w.target_ranks(), w.q, w.p, seed=0)
    for ca, cb in zip(a, b):
        assert torch.equal(ca, cb)


