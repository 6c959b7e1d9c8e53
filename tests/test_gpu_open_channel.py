"""GPU parity of the open channel (inlet, entrance grid, sponge, outlet) against the FP64 oracle.

The HIP path runs through the C ABI (lbm_set_open_channel); the oracle is
``oracle.open_channel`` started from the same state (the inlet profile at
every x with the seeded density).  Tolerances as for the periodic channel:
drag series max-norm relative error <= 1e-5, populations <= 1e-4.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import lbm as olbm
from oracle.open_channel import OpenChannel, inlet_velocity

pytestmark = pytest.mark.gpu

CM_RATES = (1.0, 1.0, 1.0)


def _ensemble(members, cap, op, collision=None, tile=None):
    from paper_2005_09323_amd.ensemble import Ensemble
    ens = Ensemble(members, series_capacity=cap)
    if tile is not None:
        ens.set_tile(tile)
    if collision is not None:
        ens.set_collision("central", *collision)
    ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau, op.outlet_rho)
    return ens


def _channel(m, op, collision=None):
    return olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square, collision,
                        open=OpenChannel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau, op.outlet_rho))


def _oracle(m, op, seed, member_index, amp, steps, collision=None):
    ch = _channel(m, op, collision)
    rho = olbm.init_density(ch, seed, member_index, amp)
    u = np.repeat(inlet_velocity(ch)[:, None], ch.nx, axis=1)
    f0 = olbm.equilibrium(rho, u, np.zeros_like(u))
    f0[:, olbm.solid_mask(ch)] = 0.0
    fout, drags = olbm.run(ch, f0, steps)
    return ch, fout, drags


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


# a 4-aligned width (row kernel) and a ragged one (per-cell kernel); grid, square and sponge in both
MEMBERS = [workloads.Member(192, 48, 0.56, 0.0, (70, 19, 8)),
           workloads.Member(130, 40, 0.6, 2e-6, (50, 16, 6))]
OPEN = workloads.OpenParams(0.05, 12, 6, 150 - 40, 0.95)  # sponge over the last ~40 / ~20 columns
OPEN_ODD = workloads.OpenParams(0.04, 9, 5, 100, 0.8)      # odd bar (half gap of 2 rows), longer sponge
OPEN_RHO = workloads.OpenParams(0.05, 12, 6, 150 - 40, 0.95, outlet_rho=1)  # outlet density extrapolated


@pytest.mark.parametrize("collision,op", [(None, OPEN), (CM_RATES, OPEN), (None, OPEN_ODD),
                                          (None, OPEN_RHO), (CM_RATES, OPEN_RHO)])
def test_open_channel_against_oracle(collision, op):
    steps = 1000
    ens = _ensemble(MEMBERS, steps, op, collision)
    assert ens.launch_steps() == 1
    ens.init(31, 1e-3)
    ens.step(steps - 1)
    torch.cuda.synchronize()
    drag = ens.drag(0, steps).cpu().numpy()
    states = [ens.state(i).double().cpu().numpy() for i in range(len(MEMBERS))]
    assert int(ens.flags().sum()) == 0
    ens.close()
    for i, m in enumerate(MEMBERS):
        ch, fout, ref = _oracle(m, op, 31, i, 1e-3, steps, collision)
        fluid = ~olbm.solid_mask(ch)
        e_drag = _rel(drag[i], ref)
        e_late = _rel(drag[i][200:], ref[200:])  # after the start-up pressure wave (drag ~50x larger)
        e_state = _rel(states[i][:, fluid], (fout - olbm.W[:, None, None])[:, fluid])
        print(f"member {i} collision {collision}: drag rel err {e_drag:.2e} (after step 200: {e_late:.2e}), "
              f"state rel err {e_state:.2e}")
        assert e_drag <= 1e-5 and e_late <= 1e-5, (i, e_drag, e_late)
        assert e_state <= 1e-4, (i, e_state)


def test_open_channel_tiles_bit_identical():
    """Every one-step launch shape gives the same states and drag; two-step shapes fall back to one step."""
    from paper_2005_09323_amd import native
    steps = 120
    runs = []
    for tile in list(range(16)) + [16, 20]:
        ens = _ensemble(MEMBERS, steps, OPEN, tile=tile)
        assert ens.launch_steps() == 1
        ens.init(5, 1e-3)
        ens.step(steps - 1)
        torch.cuda.synchronize()
        runs.append((ens.drag(0, steps).cpu().numpy(), [ens.state(i).cpu().numpy().copy() for i in range(2)]))
        ens.close()
    assert native.lib().lbm_tile_count() == 24
    d0, s0 = runs[0]
    for i, m in enumerate(MEMBERS):
        fluid = ~olbm.solid_mask(_channel(m, OPEN))
        for d, s in runs[1:]:
            assert np.array_equal(d[i], d0[i])
            assert np.array_equal(s[i][:, fluid], s0[i][:, fluid])


def test_open_channel_inactive_members_frozen():
    """Members masked off keep their state and time while the others step through the ghost kernel."""
    steps = 60
    ens = _ensemble(MEMBERS[:1] * 3, steps, OPEN)
    ens.init(9, 1e-3)
    ens.step(9)
    frozen = ens.state(1).cpu().numpy().copy()
    ens.set_active([1, 0, 1])
    ens.step(20)
    torch.cuda.synchronize()
    assert np.array_equal(ens.state(1).cpu().numpy(), frozen)
    assert [ens.time(i) for i in range(3)] == [30, 10, 30]
    ens.close()


def _golden(name):
    import os
    return np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name))


def test_paper_open_channel_sampled_members():
    """The paper's channel (512 x 128, R = 16, grid of R/2 bars, sponge), central moments, the
    full 1024-member ensemble in the launch configuration of the benchmark (two steps per
    launch): members 0, 777 and 1023 against the stored oracle series over 2000 steps, and every
    member finite."""
    wl = workloads.open_channel()
    op, rates = wl.extra["open"], wl.extra["rates"]
    steps = 2000
    ens = _ensemble(wl.members, steps, op, rates)
    assert ens.launch_steps() == 2
    ens.init(wl.seed, wl.noise_amp)
    ens.step(steps - 1)
    torch.cuda.synchronize()
    sample = (0, 777, 1023)
    drag = ens.drag(0, steps).cpu().numpy()[list(sample)]
    assert int(ens.flags().sum()) == 0
    ens.close()
    torch.cuda.empty_cache()
    for k, i in enumerate(sample):
        ref = _golden(f"open1024_m{i}_drag2000.txt")
        print(f"member {i}: drag rel err {_rel(drag[k], ref):.2e} over {steps} steps")
        assert _rel(drag[k], ref) <= 1e-5, (i, _rel(drag[k], ref))


def test_open_channel_argument_errors():
    from paper_2005_09323_amd.native import LbmError
    m = workloads.Member(192, 48, 0.56, 0.0, (70, 19, 8))
    bad = [workloads.OpenParams(0.05, 61, 8, 150, 0.9),    # grid ends next to the square's front cells
           workloads.OpenParams(0.05, 0, 6, 150, 0.9),     # grid on the inlet column
           workloads.OpenParams(-0.01, 12, 6, 150, 0.9),   # negative inlet velocity
           workloads.OpenParams(0.05, 12, 6, 150, 0.5)]    # sponge tau not above 1/2
    from paper_2005_09323_amd.ensemble import Ensemble
    ens = Ensemble([m], series_capacity=10)
    for op in bad:
        with pytest.raises(LbmError):
            ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
    ens.close()
    near_outlet = workloads.Member(192, 48, 0.56, 0.0, (182, 19, 8))  # square within 3 columns of the outlet
    ens = Ensemble([near_outlet], series_capacity=10)
    with pytest.raises(LbmError):
        ens.set_open_channel(0.05)
    ens.close()
    ens = Ensemble([m], series_capacity=10)
    for mode in (-1, 2):
        with pytest.raises(LbmError):
            ens.set_open_channel(0.05, 12, 6, 150, 0.9, outlet_density=mode)
    ens.close()
    ens = _ensemble([m], 10, OPEN)
    with pytest.raises(LbmError):
        ens.init(1, 0.0, ux0=0.02)  # an open channel starts from its inlet profile
    ens.set_open_channel(None)      # back to periodic: a uniform start is allowed again
    ens.init(1, 0.0, ux0=0.02)
    ens.close()


def test_perturbation_on_open_channel_matches_oracle():
    """Appendix-D perturbation with the mass rescale on open-channel members: the grid's bars
    are solid and stay out of every mass sum, as the square does."""
    from oracle import perturb as opert
    m = workloads.Member(64, 24, 0.56, 0.0, (30, 8, 4))
    op = workloads.OpenParams(0.05, 6, 4, 50, 0.9)
    ch = _channel(m, op)
    fluid = ~olbm.solid_mask(ch)
    assert (~fluid).sum() > 16  # the grid's bars are there

    def state(seed, steps):
        _, fout, _ = _oracle(m, op, seed, 0, 1e-2, steps)
        d = (fout - olbm.W[:, None, None]).astype(np.float32)
        d[:, ~fluid] = 0.0
        return d

    def full(d):
        f = d.astype(np.float64) + olbm.W[:, None, None]
        f[:, ~fluid] = 0.0
        return f

    n, n_snap, eps, key, period = 4, 3, 0.01, 8, 11
    states = [state(300 + i, 3) for i in range(n)]
    snaps = np.stack([state(400 + q, 5) for q in range(n_snap)])
    ens = _ensemble([m] * n, 64, op)
    ens.init(0, 0.0)
    for i in range(n):
        ens.copy_state_in(i, torch.from_numpy(states[i]).cuda(), 1)
    ens.perturb([0, 1, 0, 1], key, period, eps, torch.from_numpy(snaps).cuda())
    snaps_full = np.stack([full(snaps[q]) for q in range(n_snap)])
    for i in range(n):
        gpu = ens.state(i).double().cpu().numpy()[:, fluid]
        if i in (0, 2):
            assert np.array_equal(gpu, states[i][:, fluid].astype(np.float64))
        else:
            exp = opert.perturb(full(states[i]), snaps_full, opert.alphas(key, i, period, n_snap), eps, fluid)
            ref = (exp - olbm.W[:, None, None])[:, fluid]
            assert np.abs(gpu - ref).max() / np.abs(ref).max() <= 1e-6, i
    ens.close()


def test_gktl_run_on_open_channel_matches_oracle():
    """A GKTL run (selection, cloning, lineage rebuild, reweighted tail probability) on open-channel
    members: the ghost columns of every step come from the cloned states.  Oracle: its GKTL driving
    its open channel from the same seeded initial states."""
    import math

    from oracle import gktl as ogktl
    from paper_2005_09323_amd import rare
    m = workloads.Member(64, 24, 0.56, 0.0, (30, 8, 4))
    op = workloads.OpenParams(0.05, 6, 4, 50, 0.9)
    ch = _channel(m, op)
    n, tau, n_per, k, key, seed = 8, 16, 4, 0.5, 9, 31
    mu, sigma, dt, window = 0.0, 0.05, 1.0 / 16, 8
    ens = _ensemble([m] * n, n_per * tau + 1, op)
    ens.init(seed, 1e-2)
    ens.set_observable(mu, sigma, dt)
    run = rare.run_gktl(ens, k, n_per, tau, key)
    tr = rare.rebuild(run, ens)
    fmax = rare.window_maxima(tr.series, window)

    u = np.repeat(inlet_velocity(ch)[:, None], ch.nx, axis=1)

    def start(i):
        f0 = olbm.equilibrium(olbm.init_density(ch, seed, i, 1e-2), u, np.zeros_like(u))
        f0[:, olbm.solid_mask(ch)] = 0.0
        return olbm.collide(ch, f0)

    x0 = np.stack([start(i) for i in range(n)])

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
    ref_series = ogktl.reconstruct_series(res["samples"], res["ancestors"])
    gpu_series = tr.series.double().cpu().numpy()
    assert np.abs(gpu_series - ref_series).max() <= 1e-5 * np.abs(ref_series).max()
    lin = ogktl.lineage(res["ancestors"])
    ref_int = sum(res["integrals"][i][lin[:, i]] for i in range(n_per))
    assert np.allclose(tr.integral.cpu().numpy(), ref_int, rtol=1e-5, atol=1e-6)
    ref_fmax = ogktl.window_mean_max(ref_series, window)
    assert np.allclose(fmax.cpu().numpy(), ref_fmax, rtol=1e-5)
    ens.close()


@pytest.mark.parametrize("collision,outlet_rho", [(None, 0), (CM_RATES, 0), (None, 1), (CM_RATES, 1)])
def test_open_channel_two_step_bit_identical_to_one_step(collision, outlet_rho):
    """Widths that are multiples of 256: the two-step kernel (inlet values from the ghost block,
    the outlet ghost column of its second step built in the kernel) against the one-step shape 0,
    bit for bit; a single-strip lattice (inlet and outlet in one strip), grid bars across a strip
    seam, an odd step count, an inactive member; the oracle on the result."""
    members = [workloads.Member(512, 40, 0.56, 0.0, (200, 15, 8)),
               workloads.Member(512, 40, 0.6, 1e-6, (300, 10, 6)),
               workloads.Member(512, 40, 0.56, 0.0, (200, 15, 8))]
    op = workloads.OpenParams(0.05, 20, 6, 400, 0.9, outlet_rho)
    single = [workloads.Member(256, 33, 0.58, 0.0, (100, 12, 8))]
    op_single = workloads.OpenParams(0.04, 30, 4, 200, 0.8, outlet_rho)
    straddle = [workloads.Member(512, 40, 0.56, 0.0, (300, 15, 8))] * 2
    op_straddle = workloads.OpenParams(0.05, 252, 8, 300, 0.9, outlet_rho)  # grid bars across the strip seam
    steps = 151
    for mem, o in ((members, op), (single, op_single), (straddle, op_straddle)):
        runs = {}
        for tile in (0, 16, 17, 18, 19, 20, 21, 22, 23):  # 21-23: strips split into 128, 64, 32 rows
            ens = _ensemble(mem, steps + 40, o, collision, tile=tile)
            ens.init(41, 1e-3)
            if tile in (16, 17, 18, 19, 21, 22, 23):
                assert ens.launch_steps() == 2
            ens.step(steps - 1)
            if len(mem) > 2:
                ens.set_active([1, 0, 1])
                ens.step(33)
                ens.set_active(None)
            torch.cuda.synchronize()
            runs[tile] = ([ens.time(i) for i in range(len(mem))], ens.drag(0, steps + 33).cpu().numpy(),
                          [ens.state(i).cpu().numpy().copy() for i in range(len(mem))])
            ens.close()
        t0, d0, s0 = runs[0]
        for tile, (t, d, st) in runs.items():
            assert t == t0, tile
            for i, m in enumerate(mem):
                fluid = ~olbm.solid_mask(_channel(m, o))
                n_i = t0[i]
                assert np.array_equal(d[i][:n_i], d0[i][:n_i]), (tile, i)
                assert np.array_equal(st[i][:, fluid], s0[i][:, fluid]), (tile, i)
        m = mem[-1]
        _, _, ref = _oracle(m, o, 41, len(mem) - 1, 1e-3, steps, collision)
        assert _rel(d0[len(mem) - 1][:steps], ref) <= 1e-5



@pytest.mark.parametrize("gx0,bar", [(253, 2), (257, 3), (254, 1), (256, 4)])
def test_two_step_grid_bars_just_beyond_a_strip_seam(gx0, bar):
    """Bars ending two columns left of the strip seam at x = 256 (253 + 2) or
    starting two columns right of it (257): only the strips' outside cells
    (x = 255 and 256, collided by both neighbouring workgroups) pull from
    them, and the two-step kernel once missed them there (its grid-column
    range covered the strip's own cells only; the CPU model of its indexing
    finds that).  Bit-identical to the one-step kernel after 41 steps, both
    collisions."""
    from paper_2005_09323_amd.ensemble import Ensemble
    m = workloads.Member(512, 40, 0.56, 0.0, (400, 15, 6))
    op = workloads.OpenParams(0.04, gx0, bar, 470, 0.9)
    for collision in (None, CM_RATES):
        runs = []
        for tile in (0, 16):
            ens = Ensemble([m, m], series_capacity=60)
            ens.set_tile(tile)
            if collision is not None:
                ens.set_collision("central", *collision)
            ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
            ens.init(7, 1e-3)
            ens.step(41)
            torch.cuda.synchronize()
            runs.append((ens.drag(0, 42).cpu().numpy(), [ens.state(i).cpu().numpy().copy() for i in range(2)]))
            ens.close()
        (d0, s0), (d1, s1) = runs
        fluid = ~olbm.solid_mask(_channel(m, op))
        assert np.array_equal(d0, d1), (gx0, bar, collision)
        for i in range(2):
            assert np.array_equal(s0[i][:, fluid], s1[i][:, fluid]), (gx0, bar, collision, i)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_two_step_bounce_back_over_many_geometries(seed):
    """Bounce-back next to solid cells in the two-step kernel, for squares and grids at seeded
    random positions and sizes (across lane boundaries, strip seams and channel ends), periodic
    and open, both collisions: bit-identical to the one-step kernel after 41 steps."""
    from paper_2005_09323_amd.ensemble import Ensemble
    rng = np.random.default_rng(seed)
    for case in range(4):
        nx, ny, s = 512, int(rng.integers(20, 48)), int(rng.integers(2, 9))
        square = (int(rng.integers(24, nx - s - 4)), int(rng.integers(1, ny - s - 1)), s)
        m = workloads.Member(nx, ny, 0.56 + 0.01 * case, 0.0 if case % 2 else 2e-6, square)
        op = None
        if case % 2:
            bar = int(rng.integers(2, 7))
            op = workloads.OpenParams(0.04, int(rng.integers(2, square[0] - bar - 3)), bar,
                                      int(rng.integers(300, nx - 20)), 0.9)
        collision = CM_RATES if case >= 2 else None
        runs = []
        for tile in (0, 16):
            ens = Ensemble([m, m], series_capacity=60)
            ens.set_tile(tile)
            if collision is not None:
                ens.set_collision("central", *collision)
            if op is not None:
                ens.set_open_channel(op.u_c, op.grid_x0, op.bar, op.sponge_x0, op.sponge_tau)
            ens.init(seed * 10 + case, 1e-3)
            ens.step(41)
            torch.cuda.synchronize()
            runs.append((ens.drag(0, 42).cpu().numpy(), [ens.state(i).cpu().numpy().copy() for i in range(2)]))
            ens.close()
        (d0, s0), (d1, s1) = runs
        ch = _channel(m, op) if op is not None else olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square)
        fluid = ~olbm.solid_mask(ch)
        assert np.array_equal(d0, d1), (seed, case, square, op)
        for i in range(2):
            assert np.array_equal(s0[i][:, fluid], s1[i][:, fluid]), (seed, case, square, op, i)
