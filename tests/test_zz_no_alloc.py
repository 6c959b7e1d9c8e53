"""score_net_grad_noalloc (the score-network gradient with the library's static
workspace) against score_net_grad (the caller's workspace), through the C ABI:
the same kernels on the same inputs, so gradients and loss must agree bit for
bit.  Two calls in a row, the second with a smaller batch, so that the static
workspace still holds the first call's data when the second runs."""
import ctypes

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _inputs(batch, seed):
    p = workloads.cnn_params(seed)
    flat = np.concatenate([np.ravel(p[k]) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")])
    x, lab = workloads.cnn_batch(batch, seed + 1)
    return (torch.from_numpy(flat.astype(np.float32)).cuda(), torch.from_numpy(x.astype(np.float32)).cuda(),
            torch.from_numpy(lab.astype(np.float32)).cuda())


def _with_workspace(lib, params, x, lab):
    from paper_2005_09323_amd import native
    b = x.shape[0]
    nbytes = lib.score_net_workspace_bytes(b)
    ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device="cuda")
    g = torch.empty(lib.score_net_params(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    native.check(lib.score_net_grad(_p(params), _p(x), _p(lab), b, _p(g), _p(loss), _p(ws), nbytes, _stream()))
    return g, loss


def test_noalloc_gradient_equals_workspace_gradient_on_two_calls():
    from paper_2005_09323_amd import native
    lib = native.lib()
    runs = []
    for batch, seed in ((256, 31), (100, 41)):
        params, x, lab = _inputs(batch, seed)
        g = torch.full((lib.score_net_params(),), float("nan"), device="cuda")
        loss = torch.full((1,), float("nan"), device="cuda")
        print(f"noalloc gradient, batch {batch}, seed {seed}", flush=True)
        native.check(lib.score_net_grad_noalloc(_p(params), _p(x), _p(lab), batch, _p(g), _p(loss), _stream()))
        runs.append((params, x, lab, g.clone(), loss.clone()))
    torch.cuda.synchronize()
    for params, x, lab, g, loss in runs:
        g_ref, loss_ref = _with_workspace(lib, params, x, lab)
        torch.cuda.synchronize()
        assert torch.isfinite(g).all() and torch.isfinite(loss).all()
        assert torch.equal(g, g_ref)
        assert torch.equal(loss, loss_ref)


def test_noalloc_rejects_batches_beyond_its_workspace():
    from paper_2005_09323_amd import native
    lib = native.lib()
    params, x, lab = _inputs(4, 5)
    g = torch.empty(lib.score_net_params(), device="cuda")
    for batch in (0, 257, -1):
        rc = lib.score_net_grad_noalloc(_p(params), _p(x), _p(lab), batch, _p(g), None, _stream())
        assert rc == native.LBM_EINVAL
        assert "static workspace" in lib.lbm_last_error().decode() or batch < 1
    assert lib.score_net_grad_noalloc(None, _p(x), _p(lab), 4, _p(g), None, _stream()) == native.LBM_EINVAL
