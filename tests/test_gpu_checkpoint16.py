"""16-bit checkpoints on the GPU (FP16 / BF16 with per-field max-abs scaling).

* Against the oracle running the same schedule with the same encoding
  (``shot_gradient_checkpointed``): besides the FP32 bar (1e-5 kappa), FP32 and FP64 state
  values can straddle a 16-bit rounding boundary and flip a code; measured on MI355X the
  total stays at 1.3e-5 (FP16) and 1.9e-5 (BF16) for kappa ~ 2. Bars: 1e-5 kappa + 1e-5
  (FP16), + 2e-5 (BF16).
* Against the exact gradient (no compression): the error the encoding itself causes,
  measured 1.3e-4 (FP16) and 9e-4 (BF16) at this size (nt = 400, 20-step segments);
  stated bounds 1e-3 (FP16) and 1e-2 (BF16).
* The first forward sweep never reads a checkpoint: data are bitwise those of FP32 mode.
"""
import numpy as np
import pytest
import torch

from oracle import elastic2d as E
from test_gpu_parity2d import Case, T, _f32, kappa, rel

pytestmark = pytest.mark.gpu

MODES = {"fp16": 2, "bf16": 1}
PARITY = {"fp16": 1e-5, "bf16": 2e-5}
EXACT = {"fp16": 1e-3, "bf16": 1e-2}


@pytest.fixture(scope="module")
def ref():
    c = Case(nt=400, blob_amp=0.3)
    sh = c.sh
    c.d_obs = _f32(E.model_forward(c.grid_o, c.m_true, sh.src_iz, sh.src_ix, c.src, sh.ch_iz, sh.ch_ix))
    c.g_exact, c.phi_o, c.d_o = E.shot_gradient(c.grid_o, c.m, sh.src_iz, sh.src_ix, c.src, sh.ch_iz, sh.ch_ix,
                                                c.d_obs)
    c.kappa = kappa(c.d_o, c.d_o - c.d_obs)
    return c


@pytest.mark.parametrize("codec", ["fp16", "bf16"])
def test_compressed_checkpoints(gpu_lib, ref, codec):
    efwi = gpu_lib
    c = ref
    sh = c.sh
    L = 20
    g_same, _, _ = E.shot_gradient_checkpointed(c.grid_o, c.m, sh.src_iz, sh.src_ix, c.src, sh.ch_iz, sh.ch_ix,
                                                c.d_obs, L, codec)
    d32 = torch.empty((sh.ch_iz.size, c.grid_o.nt), dtype=torch.float32, device="cuda")
    d16 = torch.empty_like(d32)
    efwi.shot_gradient(c.grid_g(efwi), c.shot_g(efwi, ckpt_interval=L), T(c.m), T(c.src), T(c.d_obs), d_out=d32)
    g, phi = efwi.shot_gradient(c.grid_g(efwi), c.shot_g(efwi, ckpt_interval=L, ckpt_mode=MODES[codec]), T(c.m),
                                T(c.src), T(c.d_obs), d_out=d16)
    torch.cuda.synchronize()
    assert torch.equal(d32, d16)
    g = g.cpu().numpy()
    e_same = [rel(g[k], g_same[k]) for k in range(3)]
    e_exact = [rel(g[k], c.g_exact[k]) for k in range(3)]
    print(f"{codec}: vs same-encoding oracle {e_same}, vs exact {e_exact}")
    assert max(e_same) <= PARITY[codec] + 1e-5 * c.kappa, e_same
    assert max(e_exact) <= EXACT[codec], e_exact


def test_compressed_workspace_is_smaller(gpu_lib, ref):
    efwi = gpu_lib
    c = ref
    full = efwi.workspace_size(efwi.WS_GRADIENT, c.grid_g(efwi), [c.shot_g(efwi, ckpt_interval=20)])
    half = efwi.workspace_size(efwi.WS_GRADIENT, c.grid_g(efwi), [c.shot_g(efwi, ckpt_interval=20, ckpt_mode=2)])
    assert half < full
