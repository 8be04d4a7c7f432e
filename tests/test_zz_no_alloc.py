"""The allocation-free forward entry point (tsne_mlp_forward_noalloc) against
the workspace entry point (tsne_mlp_forward), through the C ABI.

Both run the same kernels; the allocation-free one keeps the BF16 weight
copies in the library's device scratch, so its output must equal the other's
bit for bit. Two calls in a row (the second with a smaller input, with other
weights) show that the scratch keeps no state that leaks from one call into
the next. Shapes and seeds are printed before each GPU step.
"""
import numpy as np
import pytest
import torch

from paper_1812_09869_amd import _lib, synth

pytestmark = pytest.mark.gpu

D, H = 50, 256


def _net(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = (rng.standard_normal(_lib.mlp_param_count(D, H)) * 0.08).astype(np.float32)
    return torch.from_numpy(p).cuda()


def test_noalloc_forward_matches_workspace_forward():
    x_np, _ = synth.gmm_aniso(5000, sample_seed=71)
    mean = torch.from_numpy(x_np.mean(axis=0).astype(np.float32)).cuda()
    invstd = torch.from_numpy((1.0 / x_np.std(axis=0)).astype(np.float32)).cuda()
    x = torch.from_numpy(x_np).cuda()
    ws = _lib.mlp_new_workspace(D, H, 1024, False)
    for n, seed in ((5000, 72), (777, 73)):
        print(f"\n[no-alloc] n={n} d_in={D} hidden={H} seed={seed}", flush=True)
        params = _net(seed)
        xs = x[:n].contiguous()
        ref = torch.empty((n, 2), device="cuda")
        _lib.mlp_forward(params, D, H, mean, invstd, xs, ref, ws)
        out = torch.full((n, 2), float("nan"), device="cuda")
        _lib.mlp_forward_noalloc(params, D, H, mean, invstd, xs, out)
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert torch.equal(out, ref), (out - ref).abs().max()
    with pytest.raises(_lib.TsneError) as e:
        _lib.mlp_forward_noalloc(params, D, 100, mean, invstd, xs, out)
    assert e.value.code == 1
