"""GPU gradient of f(X) = ||X - TT_r(X)||_F^2 through the TT-RBKI sweep (Omega fixed).

The library's reverse sweep (ttr_rbki_loss_grad) is compared with the oracle's
autograd gradient (itself pinned by finite differences of the float64 oracle sweep)
on the same stored input, and checked against central finite differences of the
library's own loss.  Shapes cover every mode kind: saturated with m <= n, regular,
saturated with n < m, identity modes and d = 2.

Tolerances: the reverse sweep repeats the forward sweep's float64 small algebra, so in
float64 the gradient agrees with the oracle's to rounding amplified by the eigen-gap
divisions (1e-8 of max |grad f|).  In float32 the streamed products carry about 1e-7
relative error of ||X|| while grad f is of the size of the residual X - Xhat (the noise
level), hence 1e-7 / noise relative error: 2e-3 for noise 1e-3 (with a factor 20 margin
for the summed products).  The loss f itself (the streamed ||X - Xhat||^2) is compared
relative to the oracle's f: 1e-8 in float64; in float32 the error eps of the sweep moves by
about 1e-7 absolute, so f = eps^2 ||X||^2 moves by 2e-7 / eps relative: 1e-3 at eps = 1e-3
(tt20x4, a factor 5 margin).

The differentiation workload (24^6, TT ranks 12, noise 1e-2, r = 12, p = 6, q = 2) runs as a
d = 6 twin against the oracle gradient and at full size against central finite differences
in float64."""
import math

import numpy as np
import pytest
import torch

import paper_2308_01480_amd as ttr
import synth
from oracle import grad as ograd
from tests.gpu_util import announce, stored_f64, to_dev

pytestmark = pytest.mark.gpu


def _small(dims, sig_rank, noise, seed):
    rng = np.random.default_rng(seed)
    X = synth.tt_full_host(synth.tt_cores_random(dims, sig_rank, 1.0, seed))
    X = X / math.sqrt(float(np.mean(X * X)))
    return X + noise * rng.standard_normal(dims)


CASES = {
    # name: (X builder, ranks, q, p)
    "tt20x4": (lambda: synth.build_host(synth.workload("tt20x4")), [5, 5, 5], 2, 5),
    "mixed5676": (lambda: _small((5, 6, 7, 6), 3, 0.3, 5), [2, 3, 2], 1, 1),
    "identity_first": (lambda: _small((3, 30, 40), 4, 1e-2, 7), [3, 4], 1, 2),
    "d2_regular": (lambda: _small((200, 300), 5, 1e-2, 9), [5], 2, 5),
    # d = 6 twin of the 24^6 differentiation workload: saturated first mode (16 x 12^5),
    # three regular modes (144 rows), a saturated last bond (n = 12 < m = 144)
    "tt24x6_twin": (lambda: synth.build_host(synth.scaled_down(synth.workload("tt24x6"), (16, 12, 12, 12, 12, 12))),
                    [12] * 5, 2, 6),
}
LOSS_TOL = {"f64": 1e-8, "f32": 1e-3}


def _compare(name, dt, rel_tol):
    build, ranks, q, p = CASES[name]
    X = build()
    announce(f"grad {name} {dt} dims={X.shape} ranks={ranks} q={q} p={p}")
    x = to_dev(X, dt)
    Xs = stored_f64(x)
    f, g = ttr.loss_grad(x, ranks, q, p, seed=0)
    torch.cuda.synchronize()
    f = float(f.cpu())
    g = g.to(torch.float64).cpu().numpy()
    fo, go = ograd.loss_and_grad(Xs, ranks, q, p, seed=0, precision=dt)
    x2 = float(np.sum(Xs * Xs))
    gmax = float(np.max(np.abs(go)))
    err = float(np.max(np.abs(g - go))) / gmax
    print(f"[gpu-case]   f_gpu={f:.12e} f_oracle={fo:.12e} max|g|={gmax:.3e} rel_grad_err={err:.3e} "
          f"rel_f_err={abs(f - fo) / fo:.3e}", flush=True)
    assert abs(f - fo) <= LOSS_TOL[dt] * fo, (name, dt, f, fo)
    assert err <= rel_tol, (name, dt, err)
    return Xs, g


@pytest.mark.parametrize("name", list(CASES))
def test_grad_matches_oracle_f64(name):
    _compare(name, "f64", 1e-8)


@pytest.mark.parametrize("name", ["tt20x4", "d2_regular", "tt24x6_twin"])
def test_grad_matches_oracle_f32(name):
    _compare(name, "f32", 2e-4 if name == "d2_regular" else 2e-3)


def test_grad_directional_fd_f64():
    build, ranks, q, p = CASES["tt20x4"]
    X = build()
    x = to_dev(X, "f64")
    _, g = ttr.loss_grad(x, ranks, q, p)
    rng = np.random.default_rng(5)
    rms = math.sqrt(float(np.mean(X * X)))
    for _ in range(3):
        D = torch.from_numpy(rng.standard_normal(X.shape)).to("cuda")
        D /= torch.linalg.norm(D)
        h = 1e-5 * rms * math.sqrt(X.size)
        fp, _ = ttr.loss_grad((x + h * D).contiguous(), ranks, q, p)
        fm, _ = ttr.loss_grad((x - h * D).contiguous(), ranks, q, p)
        fd = float((fp - fm).cpu()) / (2 * h)
        an = float(torch.sum(g * D).cpu())
        print(f"[gpu-case]   fd={fd:.10e} analytic={an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


def test_all_identity_modes_zero_loss_and_grad():
    X = np.random.default_rng(1).standard_normal((2, 3))
    x = to_dev(X, "f64")
    f, g = ttr.loss_grad(x, [2], 1, 1)
    assert abs(float(f.cpu())) <= 1e-12 * float(np.sum(X * X))
    assert float(torch.max(torch.abs(g)).cpu()) <= 1e-12


def test_autograd_function_matches_entry():
    build, ranks, q, p = CASES["mixed5676"]
    x = to_dev(build(), "f64")
    f, g = ttr.loss_grad(x, ranks, q, p, seed=3)
    xr = x.clone().requires_grad_(True)
    loss = 3.0 * ttr.rbki_loss(xr, ranks, q, p, 3)
    # forward: the plain sweep and its streamed error (no gradient work)
    f_fwd = float(ttr.rbki_loss_value(x, ranks, q, p, 3).cpu())
    assert float(loss.detach().cpu()) == 3.0 * f_fwd
    assert abs(f_fwd - float(f.cpu())) <= 1e-12 * float(f.cpu())
    loss.backward()
    # backward: the library's reverse sweep
    assert torch.equal(xr.grad, 3.0 * g)


def test_grad_coordinate_fd_f64():
    """200 coordinates of grad f on the 20^4 workload against central differences of the
    loss (h = 1e-5 RMS(X)), in float64."""
    build, ranks, q, p = CASES["tt20x4"]
    X = build()
    x = to_dev(X, "f64")
    _, g = ttr.loss_grad(x, ranks, q, p)
    g = g.cpu().numpy()
    rng = np.random.default_rng(21)
    flat = x.reshape(-1)
    idx = rng.choice(X.size, size=200, replace=False)
    h = 1e-5 * math.sqrt(float(np.mean(X * X)))
    gmax = float(np.max(np.abs(g)))
    worst = 0.0
    for i in idx:
        v = float(flat[i])
        flat[i] = v + h
        fp = float(ttr.rbki_loss_value(x, ranks, q, p).cpu())
        flat[i] = v - h
        fm = float(ttr.rbki_loss_value(x, ranks, q, p).cpu())
        flat[i] = v
        fd = (fp - fm) / (2 * h)
        worst = max(worst, abs(fd - g.reshape(-1)[i]) / gmax)
    print(f"[gpu-case]   200 coordinates: max |fd - g| / max|g| = {worst:.3e} (max|g| = {gmax:.3e})", flush=True)
    assert worst <= 1e-5


def test_grad_directional_fd_full_tt24x6_f64():
    """Central differences of f on the full-size 24^6 differentiation workload (191M entries,
    float64) along two random unit directions and one direction mixing in grad f itself."""
    w = synth.workload("tt24x6")
    x = synth.build_device(w, dtype=torch.float64)
    announce(f"grad-fd tt24x6-full dims={w.dims}")
    ranks, q, p = w.target_ranks(), w.q, w.p
    f0, g = ttr.loss_grad(x, ranks, q, p)
    gn = g / torch.linalg.norm(g)
    h = 1e-4 * math.sqrt(float(torch.mean(x * x))) * math.sqrt(x.numel())
    gen = torch.Generator(device="cuda").manual_seed(5)
    for kind in ("random", "random", "along-grad"):
        D = torch.randn(x.shape, dtype=torch.float64, device="cuda", generator=gen)
        D /= torch.linalg.norm(D)
        if kind == "along-grad":
            D = (D + gn) / torch.linalg.norm(D + gn)
        fp = float(ttr.rbki_loss_value((x + h * D).contiguous(), ranks, q, p).cpu())
        fm = float(ttr.rbki_loss_value((x - h * D).contiguous(), ranks, q, p).cpu())
        fd = (fp - fm) / (2 * h)
        an = float(torch.sum(g * D).cpu())
        print(f"[gpu-case]   {kind}: fd={fd:.10e} analytic={an:.10e} f={float(f0.cpu()):.6e}", flush=True)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (kind, fd, an)


def test_bf16_unsupported():
    x = torch.zeros((8, 8, 8), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(ttr.TTRError):
        ttr.loss_grad(x, [2, 2], 1, 1)
