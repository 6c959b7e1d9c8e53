"""GPU parity of the learned score: features, network forward/backward on BF16
matrix cores, Adam.

The network is defined with BF16 products: weights and the input of every
convolution are rounded to BF16 (nearest even), sums are FP32.  Two oracle
references, both FP64 on the same BF16-rounded weights and pictures:
* the network as defined: the oracle's forward with the input of each
  convolution rounded to BF16 too.  Outputs then differ only by FP32
  accumulation (relative L2 <= 1e-4; an FP32 emulation gives 6e-6 at batch
  256) and gradients only by the kernel's BF16 rounding of the back-propagated
  signals dZ before its matrix products (<= 5e-3 per tensor; the emulation
  gives 1.5e-3 at batch 16, 4.4e-4 at 256);
* the FP64 network without that rounding of hidden activations: outputs
  <= 1e-2, gradients <= 3e-2 per tensor.  The loose gradient bound is
  measured: ReLU masks flip where a hidden value is within a BF16 rounding of
  zero, which moves the first layer's weight gradient by 2.0e-2 at batch 16
  (w1; every other tensor <= 5.5e-3), and an emulation of the BF16 rounding
  alone reproduces those figures to two digits.
Batch 256 is the training batch of the product, whose gradient sum runs in
16 chunks of 16 images.  Features and Adam are FP32/FP64 elementwise: <= 1e-6
relative.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cnn as ocnn
from oracle import features as ofeat
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu

NAMES = ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")


def _flat(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in NAMES])


def _unflat(v):
    shp = ocnn.shapes()
    out, off = {}, 0
    for k in NAMES:
        n = int(np.prod(shp[k])) if shp[k] else 1
        out[k] = v[off:off + n].reshape(shp[k]) if shp[k] else np.array(v[off])
        off += n
    return out


def _bf16(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float64)).float().bfloat16().double().numpy()


def _bf16_params(p):
    """Weights as the matrix cores see them (BF16); biases and the read-out stay FP32."""
    q = {}
    for k in NAMES:
        v = np.asarray(p[k], dtype=np.float32).astype(np.float64)
        q[k] = _bf16(v) if k in ("w1", "w2", "w3") else v
    return q


def _net(params_flat, max_batch):
    from paper_2005_09323_amd.ensemble import ScoreNet
    return ScoreNet(torch.from_numpy(params_flat.astype(np.float32)), max_batch)


def _rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


@pytest.mark.parametrize("batch", [1, 7, 64, 256])
def test_forward_matches_oracle(batch):
    p = workloads.cnn_params(11)
    x, _ = workloads.cnn_batch(batch, 12)
    net = _net(_flat(p), batch)
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
    ref_bf16, _ = ocnn.forward(_bf16_params(p), _bf16(x.astype(np.float32)), layer_input=_bf16)
    ref, _ = ocnn.forward(_bf16_params(p), _bf16(x.astype(np.float32)))
    print(f"batch {batch} forward relative L2: {_rel_l2(y, ref_bf16):.2e} (BF16 layer inputs), "
          f"{_rel_l2(y, ref):.2e} (FP64 hidden activations)")
    assert _rel_l2(y, ref_bf16) <= 1e-4, _rel_l2(y, ref_bf16)
    assert _rel_l2(y, ref) <= 1e-2, _rel_l2(y, ref)


@pytest.mark.parametrize("batch", [16, 256])
def test_gradients_match_oracle(batch):
    p = workloads.cnn_params(21)
    x, lab = workloads.cnn_batch(batch, 22)
    net = _net(_flat(p), batch)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    lt = torch.from_numpy(lab.astype(np.float32)).cuda()
    g = net.grad(xt, lt).cpu().numpy().astype(np.float64)
    qp = _bf16_params(p)
    xb = _bf16(x.astype(np.float32))
    lab64 = lab.astype(np.float32).astype(np.float64)
    gg = _unflat(g)
    yb, cb = ocnn.forward(qp, xb, layer_input=_bf16)
    ref_bf16 = ocnn.backward(qp, cb, yb, lab64)
    y, cache = ocnn.forward(qp, xb)
    ref = ocnn.backward(qp, cache, y, lab64)
    errs_bf16 = {k: _rel_l2(gg[k], ref_bf16[k]) for k in NAMES}
    errs = {k: _rel_l2(gg[k], ref[k]) for k in NAMES}
    print(f"batch {batch} gradient relative L2 per tensor, BF16 layer inputs:",
          {k: f"{v:.2e}" for k, v in errs_bf16.items()})
    print(f"batch {batch} gradient relative L2 per tensor, FP64 hidden activations:",
          {k: f"{v:.2e}" for k, v in errs.items()})
    for k in NAMES:
        assert errs_bf16[k] <= 5e-3, (k, errs_bf16[k])
        assert errs[k] <= 3e-2, (k, errs[k])
    loss_ref = ocnn.loss(y, lab64)
    assert abs(net.loss.item() / loss_ref - 1) < 1e-2


@pytest.mark.parametrize("batch,sub,tol", [(16384, 2048, 1e-5), (4097, 2047, 2e-3)])
def test_multi_image_workgroups_match_single_image_sub_batches(batch, sub, tol):
    """From a batch of 4096 on, a backward workgroup takes several images in
    turn (8 at 16384; 2 at 4097, the last workgroup one) and sums them into one
    gradient row.  Sub-batches of at most 2047 (2048) images run one image per
    workgroup, the path pinned to the oracle above, and the batch's mean
    gradient is their mean gradients weighted by their sizes.  The kernel
    scales dZ by 1/batch before rounding it to BF16; rounding commutes with a
    power-of-two scale, so at 16384 = 8 x 2048 the two agree up to FP32
    summation order (1e-5), while at 4097 = 2047 + 2047 + 3 every BF16
    rounding of dZ lands differently: the tensors behind it (w1 .. w3) move by
    the BF16 rounding noise (<= 2e-3; measured 1.7e-4 .. 3.1e-4), the ones
    computed in FP32 throughout (b3, w4, b4) by <= 1e-5.  The forward pass is
    per image: bit-identical."""
    p = workloads.cnn_params(31)
    x, lab = workloads.cnn_batch(batch, 32)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    lt = torch.from_numpy(lab.astype(np.float32)).cuda()
    net = _net(_flat(p), batch)
    g = net.grad(xt, lt).cpu().numpy().astype(np.float64)
    loss = net.loss.item()
    y = net.forward(xt).cpu()
    subnet = _net(_flat(p), sub)
    ref = np.zeros_like(g)
    loss_ref = 0.0
    ys = []
    for s0 in range(0, batch, sub):
        s1 = min(s0 + sub, batch)
        ref += (s1 - s0) / batch * subnet.grad(xt[s0:s1].contiguous(), lt[s0:s1].contiguous()).cpu().numpy()
        loss_ref += (s1 - s0) / batch * subnet.loss.item()
        ys.append(subnet.forward(xt[s0:s1].contiguous()).cpu())
    assert torch.equal(y, torch.cat(ys))
    gg, rr = _unflat(g), _unflat(ref)
    errs = {k: _rel_l2(gg[k], rr[k]) for k in NAMES}
    print(f"batch {batch} gradient vs sub-batches of {sub}, relative L2 per tensor:",
          {k: f"{v:.1e}" for k, v in errs.items()})
    for k in NAMES:
        assert errs[k] <= (1e-5 if k in ("b3", "w4", "b4") else tol), (k, errs[k])
    assert abs(loss / loss_ref - 1) < 1e-5
    g2 = net.grad(xt, lt).cpu().numpy().astype(np.float64)
    assert np.array_equal(g, g2)  # deterministic


def test_zero_network_gives_bias_and_deterministic():
    p = {k: np.zeros_like(v) for k, v in workloads.cnn_params(0).items()}
    p["b4"] = np.array(0.375)
    x, lab = workloads.cnn_batch(5, 1)
    net = _net(_flat(p), 5)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    assert torch.all(net.forward(xt) == 0.375)
    p2 = workloads.cnn_params(3)
    net2 = _net(_flat(p2), 32)
    xb, lb = workloads.cnn_batch(32, 4)
    xt2 = torch.from_numpy(xb.astype(np.float32)).cuda()
    lt2 = torch.from_numpy(lb.astype(np.float32)).cuda()
    g1 = net2.grad(xt2, lt2).clone()
    g2 = net2.grad(xt2, lt2).clone()
    assert torch.equal(g1, g2)
    y_all = net2.forward(xt2)
    y_one = torch.cat([net2.forward(xt2[i:i + 1].contiguous()) for i in range(32)])
    assert torch.equal(y_all, y_one)


def test_adam_matches_oracle_step():
    p = workloads.cnn_params(5)
    flat = _flat(p).astype(np.float32)
    net = _net(flat.astype(np.float64), 4)
    rng = np.random.default_rng(3)
    opt = ocnn.Adam(lr=1e-3)
    ref = {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in _unflat(flat.astype(np.float64)).items()}
    for _ in range(3):
        g = rng.standard_normal(len(flat)).astype(np.float32)
        net.grads.copy_(torch.from_numpy(g))
        net.adam(lr=1e-3)
        opt.step(ref, _unflat(g.astype(np.float64)))
    got = net.params.cpu().numpy().astype(np.float64)
    assert np.abs(got - _flat(ref)).max() < 1e-6


def test_training_reduces_loss_like_oracle():
    p = workloads.cnn_params(7)
    x, _ = workloads.cnn_batch(6, 8)
    lab = 10 * x[:, 0].mean(axis=(1, 2))
    net = _net(_flat(p), 6)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    lt = torch.from_numpy(lab.astype(np.float32)).cuda()
    gpu_loss = [net.train_step(xt, lt, lr=1e-3).item() for _ in range(25)]
    ref = _bf16_params(p)
    opt = ocnn.Adam(lr=1e-3)
    ref_loss = []
    for _ in range(25):
        y, c = ocnn.forward(ref, _bf16(x.astype(np.float32)))
        ref_loss.append(ocnn.loss(y, lab))
        opt.step(ref, ocnn.backward(ref, c, y, lab))
    assert gpu_loss[-1] < 0.5 * gpu_loss[0]
    assert abs(gpu_loss[-1] / ref_loss[-1] - 1) < 0.15, (gpu_loss[-1], ref_loss[-1])


def test_features_match_oracle():
    from paper_2005_09323_amd.ensemble import Ensemble
    wl = workloads.ams_ensemble(4)
    m = wl.members[0]
    ch = olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)
    ens = Ensemble(wl.members, series_capacity=8)
    ens.init(0, 0.0)
    states = []
    for i in range(4):
        f, _ = olbm.run(ch, olbm.init_populations(ch, olbm.init_density(ch, 40 + i, 0, 1e-2)), 2)
        d = (f - olbm.W[:, None, None]).astype(np.float32)
        d[:, olbm.solid_mask(ch)] = 0
        states.append(d)
        ens.copy_state_in(i, torch.from_numpy(d).cuda(), 1)
    x0, y0, s = m.square
    px0, py0 = x0 + s - 8, y0 + s // 2 - 32  # overlaps the square's last columns
    got = ens.features(0, 4, px0, py0, 64, 4, 20.0, 200.0).cpu().numpy()
    for i in range(4):
        f = states[i].astype(np.float64) + olbm.W[:, None, None]
        f[:, olbm.solid_mask(ch)] = 0
        ref = ofeat.near_wake(ch, f, px0, py0, 64, 4, 20.0, 200.0)
        assert np.abs(got[i] - ref).max() <= 1e-6 * np.abs(ref).max() + 1e-9


def test_features_of_active_members_match_member_range():
    """score_features_active gives the rows of score_features for the active members, in
    ascending member order, bit for bit: every member at first, a subset under a mask, every
    member again after a NULL mask and after lbm_init; no rows for an empty mask; a patch
    outside an active member is rejected."""
    from paper_2005_09323_amd import native
    from paper_2005_09323_amd.ensemble import Ensemble
    m = workloads.Member(64, 32, 0.6, 1e-5, (20, 12, 6))
    n = 9
    ens = Ensemble([m] * n, series_capacity=40)
    ens.init(5, 1e-2, ux0=0.03)
    ens.step(7)
    fa = dict(px0=24, py0=0, patch=32, pool=2, u_scale=20.0, rho_scale=200.0)
    full = ens.features(0, n, **fa)
    assert torch.equal(ens.features_active(**fa), full)
    rng = np.random.default_rng(3)
    for _ in range(3):
        mask = (rng.random(n) < 0.5).astype(int)
        mask[rng.integers(n)] = 1
        ens.set_active(mask.tolist())
        got = ens.features_active(**fa)
        assert torch.equal(got, full[torch.from_numpy(np.flatnonzero(mask)).cuda()])
    ens.set_active([0] * n)
    assert ens.features_active(**fa).shape[0] == 0
    ens.set_active(None)
    assert torch.equal(ens.features_active(**fa), full)
    ens.set_active([1] + [0] * (n - 1))
    ens.init(5, 1e-2, ux0=0.03)  # every member active again, the same states as at the start
    ens.step(7)
    assert torch.equal(ens.features_active(**fa), full)
    with pytest.raises(native.LbmError):
        ens.features_active(px0=40, py0=0, patch=32, pool=2, u_scale=1.0, rho_scale=1.0)
    # an output with fewer rows than active members is refused before any write
    import ctypes
    small = torch.full((n - 1, 3, 16, 16), 7.0, device="cuda")
    rows = ctypes.c_int32()
    rc = native.lib().score_features_active(ens._ctx, 24, 0, 32, 2, 20.0, 200.0, small.data_ptr(), n - 1,
                                            ctypes.byref(rows))
    assert rc == native.LBM_EINVAL and rows.value == n
    assert bool((small == 7.0).all())
    ens.close()


def test_learned_score_predicts_future_drag_better_than_plain_score():
    """What the trained network gains over the method without it: on the stationary channel flow
    (128 members of 512 x 128 after the burn-in), the network's validation R^2 for the next
    512-step mean drag exceeds that of the plain score (the previous 512-step mean, best linear
    fit).  About 20 s on one MI355X."""
    from paper_2005_09323_amd import experiments
    _, _, _, _, rec = experiments.train_score(experiments.Flow(), 128, 100, 512, epochs=16)
    print(rec)
    assert rec["validation_r2"] > rec["plain_score_r2"] + 0.05
