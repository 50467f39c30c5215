"""Parity of the sweep at the full 48^5 benchmark size (254.8M entries) against the
float64 CPU oracle run on the same tensor (built on the GPU, copied to the host)."""
import pytest
import torch

import synth
from tests.test_gpu_sweep import run_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_size_tt48x5(dt):
    # the 48^5 benchmark workload itself (254.8M entries), oracle on the host
    w = synth.workload("tt48x5")
    x = synth.build_device(w, dtype=torch.float64)
    X = x.cpu().numpy()
    del x
    run_pair(X, w.target_ranks(), w.q, w.p, w.omega_seed, dt, "tt48x5-full")
