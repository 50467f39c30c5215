"""Parity of the sweep at the full sizes of the benchmark workloads against the float64
CPU oracle run on the same tensor (built on the GPU, copied to the host), and, for the
256^4 tensor (2^32 entries, too large for the oracle inside the test suite), the
closed-form error of its noise-free signal.

* 48^5 (254.8M entries), 24^6 (191M) and 8^10 (1.07e9): float64 and float32 sweeps against
  the oracle (eps, delta_rec, principal angles; see test_gpu_sweep.run_pair).
* 256^4 noise-free orthogonally decomposable signal sum_{i<=50} i^-1 u_i o v_i o w_i o z_i:
  every unfolding has singular values {1/i}, the rank (50) is below the Krylov width
  (q+1)(r+p) = 200, so the sweep at r = 32 reaches the TT-SVD error
  sqrt(sum_{i>32} i^-2 / sum_{i<=50} i^-2) = 0.0821427470 (stored in tests/golden with its
  derivation) in every precision: float64 and float32 to their tolerances, bfloat16 (input
  rounded to bf16, error measured against the float64 tensor) to 1%.
"""
import dataclasses
import math
import os

import pytest
import torch

import paper_2308_01480_amd as ttr
import synth
from oracle import metrics
from tests.gpu_util import announce, dev_compare
from tests.test_gpu_sweep import run_pair

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "odeco_r32_R50.txt")


def _host(w):
    x = synth.build_device(w, dtype=torch.float64)
    X = x.cpu().numpy()
    del x
    torch.cuda.empty_cache()
    return X


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_size_tt48x5(dt):
    w = synth.workload("tt48x5")
    run_pair(_host(w), w.target_ranks(), w.q, w.p, w.omega_seed, dt, "tt48x5-full")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_size_tt24x6(dt):
    w = synth.workload("tt24x6")
    run_pair(_host(w), w.target_ranks(), w.q, w.p, w.omega_seed, dt, "tt24x6-full")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_size_tt8x10(dt):
    w = synth.workload("tt8x10")
    run_pair(_host(w), w.target_ranks(), w.q, w.p, w.omega_seed, dt, "tt8x10-full", device_metrics=True)
    torch.cuda.empty_cache()


def test_full_size_odeco256x4_closed_form():
    with open(GOLDEN) as f:
        want = float(f.read().split()[0])
    w = dataclasses.replace(synth.workload("odeco256x4"), noise="none")
    announce(f"odeco256x4-full noise-free dims={w.dims} r={w.ranks} p={w.p} q={w.q}")
    x64 = synth.build_device(w, dtype=torch.float64)
    for dt, tol in (("f64", 1e-9), ("f32", 1e-6), ("bf16", 1e-2 * want)):
        x = x64 if dt == "f64" else x64.to({"f32": torch.float32, "bf16": torch.bfloat16}[dt])
        pl = ttr.plan(list(x.shape), w.ranks, w.q, w.p, x.dtype)
        assert pl.kinds == ["regular"] * 3 and list(pl.w)[:3] == [200] * 3 and bool(pl.two_pass[1])
        cores = ttr.tt_rbki(x, w.target_ranks(), w.q, w.p, seed=w.omega_seed)
        del x
        g = [c.cpu().numpy() for c in cores]
        e2, _, x2, _ = dev_compare(x64, g, g)
        eps = math.sqrt(e2 / x2)
        announce(f"odeco256x4-full {dt} eps={eps:.10e} closed_form={want:.10e}")
        assert abs(eps - want) <= tol
        assert metrics.left_orthonormality(g) <= 1e-12
        torch.cuda.empty_cache()
