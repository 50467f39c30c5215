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
for the summed products)."""
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
}


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
    print(f"[gpu-case]   f_gpu={f:.12e} f_oracle={fo:.12e} max|g|={gmax:.3e} rel_grad_err={err:.3e}", flush=True)
    assert abs(f - fo) <= max(rel_tol, 1e-12) * x2
    assert err <= rel_tol, (name, dt, err)
    return Xs, g


@pytest.mark.parametrize("name", list(CASES))
def test_grad_matches_oracle_f64(name):
    _compare(name, "f64", 1e-8)


@pytest.mark.parametrize("name", ["tt20x4", "d2_regular"])
def test_grad_matches_oracle_f32(name):
    _compare(name, "f32", 2e-3 if name == "tt20x4" else 2e-4)


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
    loss.backward()
    assert torch.equal(loss.detach(), 3.0 * f)
    assert torch.equal(xr.grad, 3.0 * g)


def test_bf16_unsupported():
    x = torch.zeros((8, 8, 8), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(ttr.TTRError):
        ttr.loss_grad(x, [2, 2], 1, 1)
