"""GPU parity of GKTL cloning, branching perturbation and AMS selection.

Selections are compared with the oracle exactly (indices, levels, branch
times): both sides take every decision in FP64 (GKTL) or on the same FP32
scores (AMS), with independent Philox implementations.  Perturbed states are
compared elementwise, relative to the largest deviation: <= 1e-6 (one FP32
rounding of values formed in FP64).
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import ams as oams
from oracle import gktl as ogktl
from oracle import lbm as olbm
from oracle import ou as oou
from oracle import perturb as opert

pytestmark = pytest.mark.gpu


def _ens(members, cap=64):
    from paper_2005_09323_amd.ensemble import Ensemble
    return Ensemble(members, series_capacity=cap)


def _channel(m):
    return olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)


def _oracle_state(m, seed, steps):
    """Post-collision populations of an oracle run (FP64) and the same as FP32 deviations."""
    ch = _channel(m)
    f, _ = olbm.run(ch, olbm.init_populations(ch, olbm.init_density(ch, seed, 0, 1e-2)), steps)
    dev32 = (f - olbm.W[:, None, None]).astype(np.float32)
    dev32[:, olbm.solid_mask(ch)] = 0.0
    return dev32


def _full(dev32, ch):
    """FP64 full populations of FP32 deviations (solid cells zero)."""
    f = dev32.astype(np.float64) + olbm.W[:, None, None]
    f[:, olbm.solid_mask(ch)] = 0.0
    return f


@pytest.mark.parametrize("n,n_bad,k,seed", [(64, 0, 1.5, 1), (64, 7, 0.3, 2), (256, 3, 4.0, 3), (1000, 0, 1.0, 4),
                                            (4096, 17, 0.7, 5), (1, 0, 1.0, 6)])
def test_gktl_selection_matches_oracle(n, n_bad, k, seed):
    """Ancestors exactly and ln R to 1e-13 against the oracle, up to the largest ensemble one
    selection handles (4096 members) and down to a single member."""
    m = workloads.Member(8, 4, 0.6, 0.0, None)
    ens = _ens([m] * n)
    ens.init(0, 0.0)
    s = workloads.log_weights(n, seed, scale=2.0, n_bad=n_bad)
    for period in range(3):
        ens.accum.copy_(torch.from_numpy(s / k))
        anc, lnr = ens.gktl_select_clone(k, key=77 + seed, period=period)
        accum_used = s / k
        ref = ogktl.select(k * accum_used, 77 + seed, period)
        assert np.array_equal(anc.cpu().numpy(), ref)
        assert math.isclose(lnr.item(), ogktl.log_normaliser(k * accum_used), rel_tol=1e-13, abs_tol=1e-13)
        assert torch.count_nonzero(ens.accum) == 0


def test_ensemble_beyond_the_selections_largest_is_rejected():
    """An ensemble holds at most the 4096 members one selection handles: a larger one is
    refused at creation."""
    from paper_2005_09323_amd import native
    m = workloads.Member(8, 4, 0.6, 0.0, None)
    with pytest.raises(native.LbmError) as e:
        _ens([m] * 4097)
    assert e.value.code == native.LBM_EINVAL


def test_gktl_all_nonfinite_is_rejected_and_changes_nothing():
    from paper_2005_09323_amd import native
    m = workloads.Member(16, 8, 0.6, 1e-5, None)
    ens = _ens([m] * 4)
    ens.init(1, 1e-3)
    before = [ens.state(i).clone() for i in range(4)]
    ens.accum.fill_(float("nan"))
    with pytest.raises(native.LbmError) as e:
        ens.gktl_select_clone(1.0, 1, 0)
    assert e.value.code == native.LBM_ENONFINITE
    for i in range(4):
        assert torch.equal(ens.state(i), before[i])


def test_gktl_clone_copies_ancestor_states_exactly():
    m = workloads.Member(64, 16, 0.6, 2e-5, (20, 5, 4))
    n = 12
    ens = _ens([m] * n)
    ens.init(5, 1e-3)
    ens.step(7)
    fluid = torch.from_numpy(~olbm.solid_mask(_channel(m))).cuda()
    before = [ens.state(i)[:, fluid].clone() for i in range(n)]
    ens.accum.copy_(torch.from_numpy(workloads.log_weights(n, 9, scale=3.0)))
    anc, _ = ens.gktl_select_clone(1.0, key=3, period=1)
    anc = anc.cpu().tolist()
    assert len(set(anc)) < n  # some trajectory was cloned, some killed
    for i in range(n):
        assert torch.equal(ens.state(i)[:, fluid], before[anc[i]])
    ens.step(5)  # the ensemble keeps running from the new states
    assert ens.time() == 13


def test_gktl_perturbation_and_mass_rescale_match_oracle():
    m = workloads.Member(64, 16, 0.56, 2e-5, (20, 5, 4))
    ch = _channel(m)
    fluid = ~olbm.solid_mask(ch)
    n, n_snap, eps, key, period = 6, 10, 0.002, 21, 4
    states = [_oracle_state(m, 100 + i, 3 + i) for i in range(n)]
    snaps = np.stack([_oracle_state(m, 200 + q, 5) for q in range(n_snap)])
    ens = _ens([m] * n)
    ens.init(0, 0.0)
    for i in range(n):
        ens.copy_state_in(i, torch.from_numpy(states[i]).cuda(), 1)
    # member 2 dominates, so it is copied several times
    s = np.array([-2.0, 0.1, 3.0, -1.0, 0.5, -0.3])
    ens.accum.copy_(torch.from_numpy(s))
    anc, _ = ens.gktl_select_clone(1.0, key=key, period=period, eps=eps,
                                   snapshots=torch.from_numpy(snaps).cuda())
    anc = anc.cpu().numpy()
    ref_anc = ogktl.select(s, key, period)
    assert np.array_equal(anc, ref_anc)
    first = ogktl.first_copy(anc)
    assert not first.all()
    snaps_full = np.stack([_full(snaps[q], ch) for q in range(n_snap)])
    for i in range(n):
        gpu = ens.state(i).double().cpu().numpy()
        parent = _full(states[anc[i]], ch)
        if first[i]:
            assert np.array_equal(gpu[:, fluid], states[anc[i]][:, fluid].astype(np.float64))
            continue
        expect = opert.perturb(parent, snaps_full, opert.alphas(key, i, period, n_snap), eps, fluid)
        ref = (expect - olbm.W[:, None, None])[:, fluid]
        err = np.abs(gpu[:, fluid] - ref).max() / np.abs(ref).max()
        assert err <= 1e-6, (i, err)
        m_gpu = math.fsum((gpu[:, fluid] + olbm.W[:, None]).ravel())
        assert abs(m_gpu / opert.total_mass(parent, fluid) - 1) < 2e-7


def test_in_place_perturbation_matches_oracle():
    m = workloads.Member(64, 16, 0.56, 2e-5, (20, 5, 4))
    ch = _channel(m)
    fluid = ~olbm.solid_mask(ch)
    n, n_snap, eps, key, period = 4, 3, 0.01, 8, 11
    states = [_oracle_state(m, 300 + i, 2) for i in range(n)]
    snaps = np.stack([_oracle_state(m, 400 + q, 4) for q in range(n_snap)])
    ens = _ens([m] * n)
    ens.init(0, 0.0)
    for i in range(n):
        ens.copy_state_in(i, torch.from_numpy(states[i]).cuda(), 1)
    ens.perturb([0, 1, 0, 1], key, period, eps, torch.from_numpy(snaps).cuda())
    snaps_full = np.stack([_full(snaps[q], ch) for q in range(n_snap)])
    for i in range(n):
        gpu = ens.state(i).double().cpu().numpy()[:, fluid]
        if i in (0, 2):
            assert np.array_equal(gpu, states[i][:, fluid].astype(np.float64))
        else:
            exp = opert.perturb(_full(states[i], ch), snaps_full, opert.alphas(key, i, period, n_snap), eps, fluid)
            ref = (exp - olbm.W[:, None, None])[:, fluid]
            assert np.abs(gpu - ref).max() / np.abs(ref).max() <= 1e-6


def test_gktl_full_ensemble_1024_gather_and_perturb():
    """256 clones of 1024 x 256: selection exact, copies exact, perturbed clones keep mass and
    are one scalar times (parent + eps sum alpha_n snapshot_n) at every sampled cell."""
    wl = workloads.gktl_ensemble()
    m = wl.members[0]
    ch = _channel(m)
    fluid_np = ~olbm.solid_mask(ch)
    fluid = torch.from_numpy(fluid_np).cuda()
    n = len(wl.members)
    eps, n_snap, key, period = 0.002, 10, 5, 2
    snaps = workloads.snapshot_states(n_snap, m, 500)
    snaps_t = torch.from_numpy(snaps).cuda()
    ens = _ens(wl.members, 300)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(20)
    before = torch.stack([ens.state(i) for i in range(n)]).clone()
    s = workloads.log_weights(n, 31, scale=1.5)
    ens.accum.copy_(torch.from_numpy(s))
    anc, _ = ens.gktl_select_clone(1.0, key=key, period=period, eps=eps, snapshots=snaps_t)
    anc = anc.cpu().numpy()
    assert np.array_equal(anc, ogktl.select(s, key, period))
    first = ogktl.first_copy(anc)
    rng = np.random.default_rng(0)
    cells = np.flatnonzero(fluid_np.ravel())[rng.integers(0, int(fluid_np.sum()), 2000)]
    snaps_full = torch.from_numpy(np.stack([_full(snaps[q], ch) for q in range(n_snap)])).cuda()
    w = torch.from_numpy(olbm.W).cuda()
    for i in range(n):
        new = ens.state(i)
        par = before[anc[i]]
        if first[i]:
            assert torch.equal(new[:, fluid], par[:, fluid])
            continue
        if i % 16:
            continue  # check a sample of the perturbed members
        al = torch.from_numpy(opert.alphas(key, i, period, n_snap)).cuda()
        f_par = par.double() + w[:, None, None]
        shifted = f_par + eps * torch.einsum("q,qiyx->iyx", al, snaps_full)
        f_new = new.double() + w[:, None, None]
        ratio = (f_new.reshape(9, -1)[:, cells] / shifted.reshape(9, -1)[:, cells])
        assert (ratio.max() - ratio.min()).item() < 1e-6
        m_new = f_new[:, fluid].sum().item()
        m_par = f_par[:, fluid].sum().item()
        assert abs(m_new / m_par - 1) < 1e-7
    ens.close()


def test_gktl_on_ou_with_device_selection():
    """The device selection drives a GKTL run of the OU process; the SCGF matches its closed form."""
    dt, steps, n_per, n, k = 0.05, 10, 10, 512, 1.0
    t_a = dt * steps * n_per
    exact = oou.log_mgf_sum(k, steps * n_per, dt) / t_a
    carrier = workloads.Member(8, 4, 0.6, 0.0, None)
    est = []
    for rep in range(4):
        ens = _ens([carrier] * n)
        ens.init(0, 0.0)
        rng = np.random.default_rng(900 + rep)
        x = oou.stationary(n, rng)
        ln_r = []
        for i in range(n_per):
            path = oou.paths(x, steps, dt, rng)
            ens.accum.copy_(torch.from_numpy(path.sum(axis=1) * dt))
            anc, lnr = ens.gktl_select_clone(k, key=rep, period=i)
            ln_r.append(lnr.item())
            x = path[anc.cpu().numpy(), -1]
        est.append(ogktl.scgf(ln_r, t_a))
        ens.close()
    mean, se = np.mean(est), np.std(est, ddof=1) / math.sqrt(len(est))
    assert abs(mean - exact) < 4 * se + 0.03 * exact, (mean, exact)


@pytest.mark.parametrize("n,t_len,n_kill,seed", [(32, 100, 1, 0), (512, 300, 26, 1), (2048, 64, 200, 2)])
def test_ams_selection_matches_oracle(n, t_len, n_kill, seed):
    from paper_2005_09323_amd.ensemble import ams_score_kill_branch
    series = workloads.score_series(n, t_len, seed)
    series[3, 10] = np.nan                       # a blown-up member
    series[5] = series[6]                        # a tie
    for it in range(3):
        res = ams_score_kill_branch(torch.from_numpy(series).cuda(), n_kill, key=40 + seed, iteration=it)
        ref = oams.kill_branch(series.astype(np.float64), n_kill, 40 + seed, it)
        assert res["level"] == ref.level
        assert np.array_equal(res["killed"].cpu().numpy(), ref.killed)
        assert np.array_equal(res["parents"].cpu().numpy(), ref.parents)
        assert np.array_equal(res["branch_t"].cpu().numpy(), ref.branch_t)
        assert np.array_equal(res["maxima"].cpu().numpy().astype(np.float64), oams.clean_maxima(series))


def test_ams_extinction():
    from paper_2005_09323_amd.ensemble import ams_score_kill_branch
    series = np.ones((8, 5), dtype=np.float32)
    res = ams_score_kill_branch(torch.from_numpy(series).cuda(), 2, key=1, iteration=0)
    assert res["n_killed"] == 8
    assert np.all(res["parents"].cpu().numpy() == -1)


def test_window_mean_score_matches_oracle():
    from paper_2005_09323_amd.ensemble import window_mean
    series = workloads.score_series(5, 400, 7)
    gpu = window_mean(torch.from_numpy(series).cuda(), 64).cpu().numpy()
    ref = ogktl.window_means(series.astype(np.float64), 64)
    assert np.all(np.isneginf(gpu[:, :63]))
    assert np.allclose(gpu[:, 63:], ref[:, 63:], rtol=2e-7, atol=1e-7)


def test_gktl_run_end_to_end_matches_oracle():
    """A whole GKTL run on the LBM ensemble (device stepping, selection, cloning, lineage
    rebuild, window maxima, reweighted tail probability) against the oracle's GKTL driving
    the oracle LBM from the same seeded initial states."""
    from paper_2005_09323_amd import rare
    m = workloads.Member(64, 16, 0.6, 2e-5, (20, 5, 4))
    ch = _channel(m)
    n, tau, n_per, k, key, seed = 8, 16, 4, 0.5, 9, 31
    mu, sigma, dt, window = 0.0, 1e-4, 1.0 / 16, 8
    ens = _ens([m] * n, cap=n_per * tau + 1)
    ens.init(seed, 1e-2)
    ens.set_observable(mu, sigma, dt)
    run = rare.run_gktl(ens, k, n_per, tau, key)
    tr = rare.rebuild(run, ens)
    fmax = rare.window_maxima(tr.series, window)

    x0 = np.stack([olbm.collide(ch, olbm.init_populations(ch, olbm.init_density(ch, seed, i, 1e-2)))
                   for i in range(n)])

    def advance(x, period):
        x = x.copy()
        samples = np.empty((n, tau))
        integ = np.empty(n)
        for j in range(n):
            fo = x[j]
            for s in range(tau):
                fo = olbm.collide(ch, olbm.stream(ch, fo))
                samples[j, s] = olbm.drag(ch, fo)
            x[j] = fo
            integ[j] = math.fsum(((samples[j] - mu) / sigma * dt).tolist())
        return x, samples, integ

    res = ogktl.run(x0, advance, n_per, k, key)
    assert np.array_equal(run.ancestors.cpu().numpy(), np.stack(res["ancestors"]))
    assert np.allclose(run.ln_r.cpu().numpy(), res["ln_r"], rtol=1e-5, atol=1e-7)
    ref_series = ogktl.reconstruct_series(res["samples"], res["ancestors"])
    gpu_series = tr.series.double().cpu().numpy()
    assert np.abs(gpu_series - ref_series).max() <= 1e-5 * np.abs(ref_series).max()
    lin = ogktl.lineage(res["ancestors"])
    ref_int = sum(res["integrals"][i][lin[:, i]] for i in range(n_per))
    assert np.allclose(tr.integral.cpu().numpy(), ref_int, rtol=1e-5, atol=1e-6)
    ref_lw = ogktl.unbias_log_weights(res["ln_r"], k, ref_int)
    assert np.allclose(tr.log_weight.cpu().numpy(), ref_lw, rtol=1e-5, atol=1e-5)
    ref_fmax = ogktl.window_mean_max(ref_series, window)
    assert np.allclose(fmax.cpu().numpy(), ref_fmax, rtol=1e-5)
    srt = np.unique(ref_fmax)
    gap = 1e-3 * (np.abs(srt).max() + 1e-30)
    # levels between distinct maxima and outside them: no ties with either side's rounding
    levels = np.concatenate([[srt[0] - gap], 0.5 * (srt[1:] + srt[:-1]), [srt[-1] + gap]])
    prob = rare.tail_probability(fmax, tr.log_weight, levels)
    ref_prob = ogktl.tail_probability(ref_fmax, ref_lw, levels)
    assert np.allclose(prob, ref_prob, rtol=1e-4)
    assert abs(run.scgf(dt) - ogktl.scgf(res["ln_r"], n_per * tau * dt)) < 1e-5 * max(1.0, abs(run.scgf(dt)))


def test_direct_sampling_estimator_matches_oracle():
    from paper_2005_09323_amd import rare
    series = workloads.score_series(6, 900, 21)
    prob, r, fmax = rare.direct_return_times(torch.from_numpy(series).cuda(), 300, 50, [0.5, 1.0, 1.5])
    blocks = series.astype(np.float64).reshape(18, 300)
    ref_fmax = ogktl.window_mean_max(blocks, 50)
    assert np.allclose(fmax.cpu().numpy(), ref_fmax, rtol=1e-6, atol=1e-7)
    ref_prob = ogktl.tail_probability(ref_fmax, np.zeros(18), np.array([0.5, 1.0, 1.5]))
    assert np.allclose(prob, ref_prob)
    assert np.allclose(r, ogktl.return_time(ref_prob, 300, 50))


def _ams_setup(n, t_a, stride, ckpt, eps, seed=17):
    from paper_2005_09323_amd import rare
    m = workloads.Member(64, 16, 0.6, 2e-5, (20, 5, 4))
    ens = _ens([m] * n, cap=t_a + 1)
    ens.init(seed, 1e-2)
    snaps = workloads.snapshot_states(3, m, 5)
    runner = rare.AmsRunner(ens, t_a, window=16, stride=stride, ckpt_every=ckpt, key=23, eps=eps,
                            snapshots=torch.from_numpy(snaps).cuda())
    return m, ens, snaps, runner


def test_ams_branch_without_perturbation_replays_parent_exactly():
    m, ens, _, runner = _ams_setup(6, 96, 8, 32, 0.0)
    res = runner.run(n_kill=2, max_iter=3, threshold=1e9)
    assert len(res.k_history) == 3
    # with eps = 0 every branch is an exact copy of its parent: each final drag series
    # equals some other member's, and the final maxima repeat
    series = ens.series[:, 1:97].cpu().numpy()
    uniq = {tuple(r.tolist()) for r in series}
    assert len(uniq) < 6
    assert res.member_steps > 6 * 96


def test_learned_ams_scores_active_members_only_bit_identical():
    """The learned-score AMS path scores only the members it steps (one feature and one forward
    pass over the active members, device-side scatter indices): bit-identical to scoring every
    member and scattering the active rows, over a run with replays, perturbations and members
    finishing at different times."""
    from paper_2005_09323_amd import rare
    from paper_2005_09323_amd.ensemble import ScoreNet

    class AllMembers(rare.AmsRunner):
        def _features(self, members, times):
            f = self.ens.features(0, self.ens.n, **self.fargs)
            y = self.net.forward(f)
            idx = torch.as_tensor(list(members), dtype=torch.long, device=self.ghat.device)
            col = torch.as_tensor(times[list(members)] // self.stride - 1, dtype=torch.long,
                                  device=self.ghat.device)
            self.ghat[idx, col] = y[idx]

    p = workloads.cnn_params(4)
    flat = np.concatenate([np.ravel(p[k]) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")])
    n, t_a, stride, ckpt = 7, 96, 8, 32
    m = workloads.Member(64, 16, 0.6, 2e-5, (20, 5, 4))
    snaps = torch.from_numpy(workloads.snapshot_states(3, m, 5)).cuda()
    fa = dict(px0=24, py0=0, patch=16, pool=1, u_scale=20.0, rho_scale=200.0)
    out = []
    for cls in (rare.AmsRunner, AllMembers):
        ens = _ens([m] * n, cap=t_a + 1)
        ens.init(31, 1e-2)
        net = ScoreNet(torch.from_numpy(flat.astype(np.float32)), n)
        runner = cls(ens, t_a, window=16, stride=stride, ckpt_every=ckpt, key=29, eps=0.01, snapshots=snaps,
                     net=net, feature_args=fa, target=0.5, width=0.1)
        res = runner.run(n_kill=2, max_iter=4, threshold=1e9)
        out.append((res.k_history, res.member_steps, runner.ghat.cpu().numpy(), ens.series[:, :t_a + 1].cpu().numpy(),
                    res.score_max))
        ens.close()
    (k_a, s_a, g_a, d_a, x_a), (k_b, s_b, g_b, d_b, x_b) = out
    assert len(k_a) == 4 and k_a == k_b and s_a == s_b
    assert np.isfinite(g_a[:, 0]).all()
    np.testing.assert_array_equal(g_a, g_b)
    np.testing.assert_array_equal(d_a, d_b)
    np.testing.assert_array_equal(x_a, x_b)


def test_ams_on_lbm_matches_oracle_ams():
    """Device AMS (checkpoints, replay, perturbation, selection) vs the oracle's AMS re-simulating
    with the oracle LBM from stored states."""
    n, t_a, stride, ckpt, eps, n_kill, iters = 5, 96, 8, 32, 0.01, 1, 3
    m, ens, snaps, runner = _ams_setup(n, t_a, stride, ckpt, eps)
    res = runner.run(n_kill=n_kill, max_iter=iters, threshold=1e9)

    ch = _channel(m)
    fluid = ~olbm.solid_mask(ch)
    snaps_full = np.stack([_full(snaps[q], ch) for q in range(3)])
    states = []   # states[j][t]: post-collision state at trajectory time t
    drags = []    # drags[j][t-1]: drag of step t
    for j in range(n):
        fo = olbm.collide(ch, olbm.init_populations(ch, olbm.init_density(ch, 17, j, 1e-2)))
        st, dr = [fo], []
        for _ in range(t_a):
            fo = olbm.collide(ch, olbm.stream(ch, fo))
            st.append(fo)
            dr.append(olbm.drag(ch, fo))
        states.append(st)
        drags.append(dr)

    def scores():
        ft = ogktl.window_means(np.array(drags), 16)
        return ft[:, stride - 1::stride]

    k_hist = []
    for it in range(iters):
        kb = oams.kill_branch(scores(), n_kill, 23, it)
        assert not kb.extinct
        k_hist.append(len(kb.killed))
        new_states, new_drags = list(states), list(drags)
        for slot, parent, tb in zip(kb.killed, kb.parents, kb.branch_t):
            t_b = (int(tb) + 1) * stride
            st = list(states[parent][:t_b + 1])
            dr = list(drags[parent][:t_b])
            fo = opert.perturb(st[t_b], snaps_full, opert.alphas(23, int(slot), it + 1, 3), eps, fluid)
            st[t_b] = fo
            for _ in range(t_b, t_a):
                fo = olbm.collide(ch, olbm.stream(ch, fo))
                st.append(fo)
                dr.append(olbm.drag(ch, fo))
            new_states[slot], new_drags[slot] = st, dr
        states, drags = new_states, new_drags
    assert res.k_history == k_hist
    ref_max = scores().max(axis=1)
    assert np.allclose(res.event_max, ref_max, rtol=1e-4, atol=1e-8)
    gpu_drag = ens.series[:, 1:t_a + 1].double().cpu().numpy()
    ref_drag = np.array(drags)
    assert np.abs(gpu_drag - ref_drag).max() <= 1e-4 * np.abs(ref_drag).max()


@pytest.mark.parametrize("level,width", [(0.0, 0.25), (1.7, 0.05), (-3.0, 1.0)])
def test_learned_score_matches_oracle_and_keeps_order(level, width):
    """ams_learned_score against the oracle's map: within one FP32 ulp of the FP64 value rounded to
    FP32, exactly the level where the event observable reached it (and nowhere else), -inf for
    non-finite predictions, never at or above the level otherwise, and predictions that
    over-shoot the level keep their order (the hard clamp tied them all)."""
    from paper_2005_09323_amd import native
    from paper_2005_09323_amd.ensemble import _ptr, _stream_handle
    rng = np.random.default_rng(11)
    n = 40_000
    ghat = (level + width * rng.uniform(-30.0, 12.0, n)).astype(np.float32)
    ghat[:5] = [np.nan, np.inf, -np.inf, level, np.float32(level) + 10 * width]
    ft = (level + width * rng.uniform(-5.0, 1.0, n)).astype(np.float32)
    ft[:5] = level - 1.0
    ft[5] = level                               # the event reached exactly at the level
    g, f = torch.from_numpy(ghat).cuda(), torch.from_numpy(ft).cuda()
    out = torch.empty_like(g)
    native.check(native.lib().ams_learned_score(_ptr(g), _ptr(f), n, level, width, _ptr(out),
                                                _stream_handle(None)))
    got = out.cpu().numpy()
    ref = oams.learned_score(ghat.astype(np.float64), ft.astype(np.float64), float(np.float32(level)),
                             float(np.float32(width)))
    lev32 = np.float32(level)
    hit = ft >= lev32
    assert np.array_equal(got == lev32, hit)
    assert np.all(got[~hit] < lev32)
    assert got[0] == -np.inf and got[1] == -np.inf and got[2] == -np.inf
    fin = np.isfinite(ref) & ~hit
    ref32 = np.minimum(ref[fin].astype(np.float32), np.nextafter(lev32, np.float32(-np.inf)))
    ulp = np.spacing(np.abs(ref32)).astype(np.float64)
    assert np.all(np.abs(got[fin].astype(np.float64) - ref32.astype(np.float64)) <= ulp), \
        np.max(np.abs(got[fin].astype(np.float64) - ref32) / ulp)
    # order: monotone everywhere, and strictly increasing on a grid from the level up to 8 widths
    # above it (FP32 resolves the approach that far)
    order = np.argsort(ghat[fin], kind="stable")
    assert np.all(np.diff(got[fin][order]) >= 0)
    grid = (lev32 + np.float32(width) * np.arange(0, 8.01, 0.5, dtype=np.float32)).astype(np.float32)
    gg, ff = torch.from_numpy(grid).cuda(), torch.full((grid.size,), -np.inf, device="cuda")
    og = torch.empty_like(gg)
    native.check(native.lib().ams_learned_score(_ptr(gg), _ptr(ff), grid.size, level, width, _ptr(og),
                                                _stream_handle(None)))
    assert np.all(np.diff(og.cpu().numpy()) > 0)


def test_learned_score_argument_errors():
    from paper_2005_09323_amd import native
    from paper_2005_09323_amd.ensemble import _ptr, _stream_handle
    g = torch.zeros(4, device="cuda")
    for level, width in ((float("nan"), 1.0), (1.0, 0.0), (1.0, -1.0), (1.0, float("inf"))):
        rc = native.lib().ams_learned_score(_ptr(g), _ptr(g), 4, level, width, _ptr(g), _stream_handle(None))
        assert rc == native.LBM_EINVAL


@pytest.mark.parametrize("eps,n_snap", [(0.002, 10), (0.0, 0)])
def test_relabelling_clone_bit_identical_to_gather(eps, n_snap):
    """GKTL cloning by relabelling member blocks (the default: the first copy of an ancestor moves
    no data) against gathering every copy into the other buffer: ancestors, states, drag series and
    integrals bit for bit over six periods of 128 steps (two-step kernel, graph replays), with the
    perturbation and with eps = 0 (further copies are plain copies).  The members' blocks stay a
    permutation of the canonical ones."""
    m = workloads.Member(256, 32, 0.56, 2e-5, (60, 12, 8))
    n, tau, periods = 48, 128, 6
    snaps = torch.from_numpy(workloads.snapshot_states(max(n_snap, 1), m, 3)).cuda()[:n_snap].contiguous()
    runs = {}
    for relabel in (True, False):
        ens = _ens([m] * n, cap=tau * periods + 10)
        ens.set_tile(16)  # two steps per launch over whole strips
        ens.set_cloning(relabel)
        ens.init(17, 1e-2)
        ens.set_observable(0.0, 1e-4, 1.0 / 64)
        ancs, ints = [], []
        for p in range(periods):
            ens.step(tau)
            ints.append(ens.accum.clone())
            anc, _ = ens.gktl_select_clone(1.0, key=5, period=p, eps=eps, snapshots=snaps if n_snap else None)
            ancs.append(anc.clone())
        ens.step(7)  # an odd step after the last clone
        torch.cuda.synchronize()
        fluid = torch.from_numpy(~olbm.solid_mask(_channel(m))).cuda()
        ptrs = sorted(ens.state(i).data_ptr() for i in range(n))
        runs[relabel] = (torch.stack(ancs).cpu(), torch.stack(ints).cpu(), ens.drag(0, ens.time()).cpu(),
                         torch.stack([ens.state(i)[:, fluid] for i in range(n)]).cpu(), ptrs, ens)
    a1, i1, d1, s1, p1, e1 = runs[True]
    a0, i0, d0, s0, p0, e0 = runs[False]
    assert len(set(a1[0].tolist())) < n            # lineages were cut and copied
    assert torch.equal(a1, a0) and torch.equal(i1, i0)
    assert torch.equal(d1, d0) and torch.equal(s1, s0)
    # every block in use exactly once (offsets within a buffer are a permutation)
    floats = 9 * m.nx * m.ny
    for ens, ptrs in ((e1, p1), (e0, p0)):
        offs = sorted(((p - ens.pop_a.data_ptr()) if ens.pop_a.data_ptr() <= p < ens.pop_a.data_ptr() + ens.pop_a.numel() * 4
                       else (p - ens.pop_b.data_ptr())) // 4 for p in ptrs)
        assert offs == [k * floats for k in range(n)]
    e1.close()
    e0.close()


def test_estimators_in_fp64_on_the_device_match_oracle():
    """The SCGF of a GKTL run, return times from probabilities, and the unbiased AMS estimate,
    computed by the library in FP64, against the oracle's definitions (Appendix C.1, C.2, B):
    seeded inputs plus the edge cases (one period, probabilities 0 and 1, no AMS iteration,
    levels above and below every maximum); argument errors leave the outputs alone."""
    from paper_2005_09323_amd import native
    from paper_2005_09323_amd.ensemble import _ptr, _stream_handle
    lib = native.lib()
    st = _stream_handle(None)
    rng = np.random.default_rng(41)
    for n_periods in (1, 7, 300):
        ln_r = rng.normal(0.3, 2.0, n_periods)
        d = torch.tensor(ln_r, dtype=torch.float64, device="cuda")
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        t_a = 16.0 * n_periods * 0.25
        native.check(lib.gktl_scgf(_ptr(d), n_periods, t_a, _ptr(out), st))
        ref = ogktl.scgf(ln_r, t_a)
        assert abs(out.item() - ref) <= 1e-13 * max(1.0, abs(ref)), n_periods
    probs = np.concatenate([[0.0, 1e-300, 1e-12, 1e-6, 0.3, 0.999, 1.0], rng.uniform(0, 1, 40)])
    p = torch.tensor(probs, dtype=torch.float64, device="cuda")
    r = torch.empty_like(p)
    for t_a, window in ((300.0, 50.0), (40.0, 0.0)):
        native.check(lib.return_times(_ptr(p), len(probs), t_a, window, _ptr(r), st))
        got = r.cpu().numpy()
        with np.errstate(divide="ignore"):  # p = 1 in the oracle: ln 0
            ref = ogktl.return_time(probs, t_a, window) if window else oams.return_time(probs, t_a)
        assert np.isinf(got[0]) and got[6] == 0.0
        assert np.allclose(got[1:], ref[1:], rtol=1e-14, atol=0.0), (t_a, window)
    for bad in ((40.0, 40.0), (40.0, -1.0), (math.inf, 0.0)):
        r.fill_(7.0)
        assert lib.return_times(_ptr(p), len(probs), bad[0], bad[1], _ptr(r), st) != 0
        assert torch.all(r == 7.0)
    assert lib.return_times(None, 0, 10.0, 1.0, None, st) == 0
    for n, n_iter in ((512, 0), (512, 26), (37, 5)):
        kh = rng.integers(1, max(2, n // 10), n_iter).astype(np.int32)
        final = rng.normal(0.0, 1.0, n)
        levels = np.concatenate([[final.min() - 1, final.max() + 1, final.max()], np.quantile(final, [0.1, 0.5, 0.9])])
        khd = torch.tensor(kh, dtype=torch.int32, device="cuda")
        fd = torch.tensor(final, dtype=torch.float64, device="cuda")
        ld = torch.tensor(levels, dtype=torch.float64, device="cuda")
        pd = torch.empty_like(ld)
        native.check(lib.ams_probability(_ptr(khd) if n_iter else None, n_iter, n, _ptr(fd), _ptr(ld), len(levels),
                                         _ptr(pd), st))
        ref = oams.estimate(list(kh), n, final, levels)
        assert np.allclose(pd.cpu().numpy(), ref, rtol=1e-14, atol=0.0), (n, n_iter)
        assert pd[1].item() == 0.0
    assert lib.ams_probability(None, 3, 10, _ptr(fd), _ptr(ld), len(levels), _ptr(pd), st) != 0
    assert lib.ams_probability(_ptr(khd), 1, 0, _ptr(fd), _ptr(ld), len(levels), _ptr(pd), st) != 0
    assert lib.gktl_scgf(_ptr(fd), 0, 1.0, _ptr(pd), st) != 0
    assert lib.gktl_scgf(_ptr(fd), 3, 0.0, _ptr(pd), st) != 0
