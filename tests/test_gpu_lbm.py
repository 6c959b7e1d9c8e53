"""GPU parity of the lattice-Boltzmann hot path against the FP64 oracle.

Every test runs the HIP kernels through the C ABI and compares with the
oracle on the same seeded inputs.  Tolerances:
* drag series: max_t |f_gpu - f_orc| / max_t |f_orc| <= 1e-5 (FP32 storage and
  arithmetic against FP64; relative per-sample error is undefined where the
  drag crosses zero);
* populations: the same max-norm relative error <= 1e-4 (FP32 round-off of
  O(1e-7) per step, accumulated over up to 2000 steps of a weakly damped flow).
"""
import os

import numpy as np
import pytest
import torch

import workloads
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ensemble(members, cap):
    from paper_2005_09323_amd.ensemble import Ensemble
    return Ensemble(members, series_capacity=cap)


def _channel(m, collision=None):
    return olbm.Channel(m.nx, m.ny, m.tau, m.force_x, m.square, collision)


def _oracle(m, seed, member_index, amp, steps, collision=None, ux0=0.0):
    ch = _channel(m, collision)
    f0 = olbm.init_populations(ch, olbm.init_density(ch, seed, member_index, amp), ux0)
    return olbm.run(ch, f0, steps)


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def _state_err(ens, idx, m, fout):
    ch = _channel(m)
    fluid = ~olbm.solid_mask(ch)
    gpu = ens.state(idx).double().cpu().numpy()
    ref = fout - olbm.W[:, None, None]
    return _rel(gpu[:, fluid], ref[:, fluid])


def test_single_channel_2000_steps():
    """256 x 64 channel, square 8, tau 0.55, g 1e-6, 2000 steps (the single-trajectory workload)."""
    wl = workloads.single_channel()
    m = wl.members[0]
    ens = _ensemble([m], wl.steps)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(wl.steps - 1)
    gpu = ens.drag(0, wl.steps).cpu().numpy()[0]
    fout, ref = _oracle(m, wl.seed, 0, wl.noise_amp, wl.steps)
    print("drag rel err", _rel(gpu, ref), "state rel err", _state_err(ens, 0, m, fout))
    assert _rel(gpu, ref) <= 1e-5
    assert _state_err(ens, 0, m, fout) <= 1e-4


def test_ragged_mixed_shapes_all_tiles():
    """Several shapes in one launch, sizes not multiples of any tile, every tile shape bit-identical."""
    members = [workloads.Member(200, 37, 0.6, 2e-5, (50, 10, 6)),
               workloads.Member(200, 37, 0.53, 1e-5, (120, 20, 5)),
               workloads.Member(64, 16, 0.7, 4e-5, None),
               workloads.Member(130, 21, 0.56, 3e-5, (1, 1, 3))]
    steps = 300
    from paper_2005_09323_amd import native
    results = []
    for tile in range(native.lib().lbm_tile_count()):
        ens = _ensemble(members, steps)
        ens.set_tile(tile)
        ens.init(11, 1e-2)
        ens.step(steps - 1)
        torch.cuda.synchronize()
        results.append((ens.drag(0, steps).cpu().numpy(), [ens.state(i).cpu().numpy().copy() for i in range(4)]))
        ens.close()
    drag0, states0 = results[0]
    for i, m in enumerate(members):
        fout, ref = _oracle(m, 11, i, 1e-2, steps)
        fluid = ~olbm.solid_mask(_channel(m))
        if m.square is not None:
            assert _rel(drag0[i], ref) <= 1e-5, i
        else:
            assert np.all(drag0[i] == 0)
        err = _rel(states0[i][:, fluid], (fout - olbm.W[:, None, None])[:, fluid])
        assert err <= 1e-4, (i, err)
    for drag, states in results[1:]:
        assert np.array_equal(drag, drag0)
        for i, m in enumerate(members):
            fluid = ~olbm.solid_mask(_channel(m))
            assert np.array_equal(states[i][:, fluid], states0[i][:, fluid])


def _two_step_tiles():
    from paper_2005_09323_amd import native
    lib = native.lib()
    # 20 is the adaptive default; 21-23 split every strip into workgroups of 128, 64 and 32 rows
    return [t for t in range(16, lib.lbm_tile_count()) if t != 20]


def test_two_step_shapes_bit_identical_to_one_step():
    """Widths that are multiples of 256: the two-step kernel (every shape) against shape 0, bit for bit.

    Squares straddling a strip boundary and next to the periodic edges, a lattice lower than
    the rows per iteration, and an odd step count (chunks that end with a single step); strips
    split into row ranges, with a square across the seams at rows 64 and 128."""
    members = [workloads.Member(256, 37, 0.6, 2e-5, (50, 10, 6)),
               workloads.Member(256, 150, 0.57, 2e-5, (100, 60, 8)),
               workloads.Member(256, 150, 0.57, 2e-5, (200, 124, 8)),
               workloads.Member(512, 21, 0.53, 1e-5, (253, 8, 6)),
               workloads.Member(256, 12, 0.56, 3e-5, (1, 1, 3)),
               workloads.Member(256, 12, 0.56, 3e-5, (251, 7, 4)),
               workloads.Member(768, 5, 0.7, 4e-5, None),
               workloads.Member(256, 16, 0.52, 1e-5, (120, 5, 6))]
    steps = 301
    results = {}
    for tile in [0] + _two_step_tiles():
        ens = _ensemble(members, steps)
        ens.set_tile(tile)
        ens.init(13, 1e-2)
        ens.step(steps - 1)
        torch.cuda.synchronize()
        results[tile] = (ens.drag(0, steps).cpu().numpy(),
                         [ens.state(i).cpu().numpy().copy() for i in range(len(members))],
                         [ens.time(i) for i in range(len(members))])
        ens.close()
    drag0, states0, times0 = results[0]
    assert times0 == [steps] * len(members)
    for i, m in enumerate(members):
        if m.square is None:
            assert np.all(drag0[i] == 0)
            continue
        fout, ref = _oracle(m, 13, i, 1e-2, steps)
        assert _rel(drag0[i], ref) <= 1e-5, i
    for tile, (drag, states, times) in results.items():
        assert times == times0, tile
        assert np.array_equal(drag, drag0), tile
        for i, m in enumerate(members):
            fluid = ~olbm.solid_mask(_channel(m))
            assert np.array_equal(states[i][:, fluid], states0[i][:, fluid]), (tile, i)


def test_two_step_with_inactive_members_and_odd_batches():
    """Per-member stepping (set_active) and batches of 1, 2 and 63 steps on the two-step shape."""
    m = workloads.Member(512, 40, 0.55, 2e-5, (100, 15, 8))
    runs = []
    for tile in (0, _two_step_tiles()[0]):
        ens = _ensemble([m] * 3, 400)
        ens.set_tile(tile)
        ens.init(21, 1e-2)
        ens.step(1)
        ens.set_active([1, 0, 1])
        ens.step(2)
        ens.step(63)
        ens.set_active(None)
        ens.step(65)
        torch.cuda.synchronize()
        runs.append(([ens.time(i) for i in range(3)], ens.drag(0, 132).cpu().numpy(),
                     [ens.state(i).cpu().numpy().copy() for i in range(3)]))
        ens.close()
    (t0, d0, s0), (t1, d1, s1) = runs
    assert t0 == t1 == [132, 67, 132]
    assert np.array_equal(d0[[0, 2]], d1[[0, 2]]) and np.array_equal(d0[1, :67], d1[1, :67])
    fluid = ~olbm.solid_mask(_channel(m))
    for i in range(3):
        assert np.array_equal(s0[i][:, fluid], s1[i][:, fluid]), i


CM_RATES = (1.0, 1.0, 1.0)  # bulk, third-order and fourth-order rates of the central-moment collision


@pytest.mark.parametrize("rates", [CM_RATES, (1.3, 0.8, 1.6)])
def test_central_moments_against_oracle_both_kernels(rates):
    """Central-moment collision against the oracle's, on one-step and two-step launches (bit-identical)."""
    members = [workloads.Member(256, 37, 0.52, 2e-5, (60, 12, 8)),
               workloads.Member(512, 24, 0.505, 1e-5, (250, 8, 6))]
    steps = 401
    results = {}
    for tile in (0, _two_step_tiles()[0]):
        ens = _ensemble(members, steps)
        ens.set_tile(tile)
        ens.set_collision("central", *rates)
        ens.init(17, 1e-2)
        ens.step(steps - 1)
        torch.cuda.synchronize()
        results[tile] = (ens.drag(0, steps).cpu().numpy(), [ens.state(i).cpu().numpy().copy() for i in range(2)])
        ens.close()
    (d0, s0), (d1, s1) = results.values()
    assert np.array_equal(d0, d1)
    for i, m in enumerate(members):
        fluid = ~olbm.solid_mask(_channel(m))
        assert np.array_equal(s0[i][:, fluid], s1[i][:, fluid]), i
        fout, ref = _oracle(m, 17, i, 1e-2, steps, collision=rates)
        assert _rel(d0[i], ref) <= 1e-5, (i, _rel(d0[i], ref))
        assert _rel(s0[i][:, fluid], (fout - olbm.W[:, None, None])[:, fluid]) <= 1e-4


def test_central_moments_impulsive_start_near_half():
    """tau = 0.5005, uniform flow started impulsively around the square: bounded, and equal to the oracle."""
    m = workloads.Member(256, 32, 0.5005, 0.0, (30, 13, 6))
    steps = 300
    ens = _ensemble([m], 700)
    ens.set_collision("central", *CM_RATES)
    ens.init(0, 0.0, ux0=0.08)
    ens.step(steps - 1)
    torch.cuda.synchronize()
    gpu = ens.drag(0, steps).cpu().numpy()[0]
    fout, ref = _oracle(m, 0, 0, 0.0, steps, collision=CM_RATES, ux0=0.08)
    assert _rel(gpu, ref) <= 1e-5
    ens.step(400)
    assert int(ens.flags().sum()) == 0
    assert bool(torch.isfinite(ens.drag(0, 700)).all())
    ens.close()


def test_collision_argument_errors():
    m = workloads.Member(256, 16, 0.6, 1e-5, None)
    ens = _ensemble([m], 10)
    from paper_2005_09323_amd.native import LbmError
    for bad in ((1, 0.0, 1.0, 1.0), (1, 1.0, 2.0, 1.0), (2, 1.0, 1.0, 1.0)):
        with pytest.raises(LbmError):
            from paper_2005_09323_amd import native
            native.check(native.lib().lbm_set_collision(ens._ctx, *bad))
    ens.set_collision("bgk")
    ens.close()


def test_adaptive_default_shape():
    """The default shape makes two steps per launch while the active members fill the device and
    one step otherwise; either way the states equal those of the one-step shape 0."""
    wl = workloads.ensemble_1024()
    few = [1] * 8 + [0] * (len(wl.members) - 8)
    runs = []
    for tile in (None, 0):
        ens = _ensemble(wl.members, 20)
        if tile is not None:
            ens.set_tile(tile)
        ens.init(wl.seed, wl.noise_amp)
        if tile is None:
            assert ens.launch_steps() == 2
        ens.step(4)
        ens.set_active(few)
        if tile is None:
            assert ens.launch_steps() == 1
        ens.step(5)
        ens.set_active(None)
        ens.step(3)
        torch.cuda.synchronize()
        runs.append(([ens.time(i) for i in (0, 8)], ens.drag(0, 13).cpu().numpy()[[0, 7, 8, 127]],
                     [ens.state(i).cpu().numpy().copy() for i in (0, 8)]))
        ens.close()
        torch.cuda.empty_cache()
    (t0, d0, s0), (t1, d1, s1) = runs
    assert t0 == t1 == [13, 8]
    assert np.array_equal(d0[:, :8], d1[:, :8]) and np.array_equal(d0[:2], d1[:2])
    fluid = ~olbm.solid_mask(_channel(wl.members[0]))
    for a, b in zip(s0, s1):
        assert np.array_equal(a[:, fluid], b[:, fluid])


def test_face_diagnostics_against_oracle():
    """Pressure, stress-integral drag and shear on the square's faces after a noisy forced run
    (both collisions), against the oracle's on its own run."""
    from oracle import diagnostics as odg
    members = [workloads.Member(256, 37, 0.52, 2e-5, (60, 12, 8)),
               workloads.Member(256, 37, 0.6, 1e-5, (120, 20, 5)),
               workloads.Member(256, 37, 0.6, 1e-5, None)]
    steps = 300
    for collision in (None, CM_RATES):
        ens = _ensemble(members, steps)
        if collision is not None:
            ens.set_collision("central", *collision)
        ens.init(23, 1e-2)
        ens.step(steps - 1)
        gpu = ens.face_diagnostics().cpu().numpy()
        ens.close()
        for i, m in enumerate(members):
            ch = _channel(m, collision)
            fout, _ = _oracle(m, 23, i, 1e-2, steps, collision=collision)
            ref = odg.diagnostics(ch, olbm.stream(ch, fout))
            if m.square is None:
                assert np.all(gpu[i] == 0)
                continue
            scale = np.array([ref[0], ref[0], abs(ref[2]), abs(ref[3]), abs(ref[4])])
            assert np.all(np.abs(gpu[i] - ref) <= 1e-5 * scale), (i, gpu[i], ref)


def test_rest_state_exact_and_deterministic():
    m = workloads.Member(256, 64, 0.51, 0.0, (60, 28, 8))
    ens = _ensemble([m, m], 50)
    ens.init(1, 0.0)
    ens.step(49)
    fluid = torch.from_numpy(~olbm.solid_mask(_channel(m))).cuda()
    for i in range(2):
        assert torch.count_nonzero(ens.state(i)[:, fluid]) == 0
    assert torch.count_nonzero(ens.drag(0, 50)) == 0


def test_run_twice_bit_identical_and_mass_conserved():
    m = workloads.Member(512, 128, 0.52, 2e-6, (120, 56, 16))
    runs = []
    for _ in range(2):
        ens = _ensemble([m] * 3, 400)
        ens.init(5, 1e-3)
        fluid = torch.from_numpy(~olbm.solid_mask(_channel(m))).cuda()
        mass0 = [ens.state(i)[:, fluid].double().sum().item() for i in range(3)]
        ens.step(399)
        mass1 = [ens.state(i)[:, fluid].double().sum().item() for i in range(3)]
        runs.append((ens.drag(0, 400).cpu(), torch.stack([ens.state(i) for i in range(3)]).cpu()))
        ens.close()
        n_fluid = int(fluid.sum())
        for a, b in zip(mass0, mass1):
            assert abs(a - b) <= 1e-6 * n_fluid  # FP32 round-off of O(1e-8) per cell
    assert torch.equal(runs[0][0], runs[1][0])
    mask = ~olbm.solid_mask(_channel(m))
    assert np.array_equal(runs[0][1].numpy()[:, :, mask], runs[1][1].numpy()[:, :, mask])


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name))


@pytest.mark.parametrize("member,name", [(0, "ensemble1024_m0_drag1000.txt"),
                                         (127, "ensemble1024_m127_drag1000.txt")])
def test_full_ensemble_1024_against_stored_oracle(member, name):
    """128 x 1024 x 256 (tau 0.5015, g 3e-6): the whole ensemble in one launch, members checked on 1000 steps."""
    wl = workloads.ensemble_1024()
    ens = _ensemble(wl.members, 1000)
    ens.autotune(6)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(999)
    gpu = ens.drag(0, 1000).cpu().numpy()
    ref = _golden(name)
    assert _rel(gpu[member], ref) <= 1e-5
    ens.close()


def test_full_ensemble_1024_two_step_against_stored_oracle():
    """The two-step kernel on the whole 128 x 1024 x 256 ensemble, members 0 and 127, 1000 steps."""
    wl = workloads.ensemble_1024()
    ens = _ensemble(wl.members, 1000)
    ens.set_tile(_two_step_tiles()[0])
    ens.init(wl.seed, wl.noise_amp)
    ens.step(999)
    gpu = ens.drag(0, 1000).cpu().numpy()
    assert _rel(gpu[0], _golden("ensemble1024_m0_drag1000.txt")) <= 1e-5
    assert _rel(gpu[127], _golden("ensemble1024_m127_drag1000.txt")) <= 1e-5
    assert int(ens.flags().sum()) == 0
    ens.close()


def test_mixed_sizes_against_stored_oracle():
    wl = workloads.mixed_sizes()
    ens = _ensemble(wl.members, 1000)
    ens.init(wl.seed, wl.noise_amp)
    ens.step(999)
    gpu = ens.drag(0, 1000).cpu().numpy()
    for idx, name in ((0, "mixed_m0_drag1000.txt"), (64, "mixed_m64_drag1000.txt"),
                      (191, "mixed_m191_drag1000.txt")):
        assert _rel(gpu[idx], _golden(name)) <= 1e-5, idx
    ens.close()


def test_inactive_members_are_frozen_and_resume_exactly():
    m = workloads.Member(128, 32, 0.6, 1e-5, (30, 12, 6))
    ref = _ensemble([m, m], 120)
    ref.init(3, 1e-3)
    ref.step(100)
    ens = _ensemble([m, m], 120)
    ens.init(3, 1e-3)
    ens.step(40)
    ens.set_active([1, 0])
    snap = ens.state(1).clone()
    ens.step(60)
    assert ens.time(0) == 101 and ens.time(1) == 41
    assert torch.equal(ens.state(1), snap)
    ens.set_active([0, 1])
    ens.step(60)
    ens.set_active(None)
    fluid = torch.from_numpy(~olbm.solid_mask(_channel(m))).cuda()
    for i in range(2):
        assert torch.equal(ens.state(i)[:, fluid], ref.state(i)[:, fluid])
    assert torch.equal(ens.drag(0, 101), ref.drag(0, 101))


def test_nonfinite_member_is_flagged_and_isolated():
    m = workloads.Member(128, 32, 0.6, 1e-5, (30, 12, 6))
    ens = _ensemble([m] * 3, 60)
    ens.init(2, 1e-3)
    ens.state(1)[:, 14, 40] = float("nan")  # four cells from the square
    ens.step(30)
    flags = ens.flags().cpu().tolist()
    assert flags == [0, 1, 0]
    ref = _ensemble([m] * 3, 60)
    ref.init(2, 1e-3)
    ref.step(30)
    assert torch.equal(ens.drag(0, 31)[0], ref.drag(0, 31)[0])
    assert torch.equal(ens.drag(0, 31)[2], ref.drag(0, 31)[2])


def test_capacity_and_argument_errors():
    from paper_2005_09323_amd import native
    m = workloads.Member(64, 16, 0.6, 1e-5, None)
    ens = _ensemble([m], 10)
    ens.init(1, 0.0)
    ens.step(9)
    with pytest.raises(native.LbmError) as e:
        ens.step(1)
    assert e.value.code == native.LBM_ERANGE
    with pytest.raises(native.LbmError):
        ens.set_tile(999)
    ens.set_time(1)
    ens.step(3)
    assert ens.time() == 4
    assert ens.drag(2, 2).shape == (1, 0)  # an empty column range copies nothing
    with pytest.raises(native.LbmError):
        ens.drag(0, 11)  # beyond the series capacity


def test_init_with_uniform_velocity_matches_oracle():
    m = workloads.Member(512, 128, 0.502, 9e-7, workloads.centred_square(128, 64, 16))
    steps = 400
    ens = _ensemble([m, m], steps)
    ens.init(8, 1e-3, ux0=0.05)
    ens.step(steps - 1)
    gpu = ens.drag(0, steps).cpu().numpy()
    for i in range(2):
        ch = _channel(m)
        f0 = olbm.init_populations(ch, olbm.init_density(ch, 8, i, 1e-3), ux0=0.05)
        fout, ref = olbm.run(ch, f0, steps)
        assert _rel(gpu[i], ref) <= 1e-5
        assert _state_err(ens, i, m, fout) <= 1e-4


def test_autotune_table_is_reused(tmp_path):
    """A tuned shape goes into the table under the ensemble's key, a new context with that key
    reads it back, and a different collision is a different key (tuned and appended)."""
    from paper_2005_09323_amd.ensemble import Ensemble
    members = [workloads.Member(512, 64, 0.6, 1e-5, (100, 20, 8))] * 8
    table = str(tmp_path / "tiles.txt")
    ens = Ensemble(members, series_capacity=10)
    t1 = ens.autotune(4, table=table)
    ens.close()
    lines = open(table).read().splitlines()
    assert len(lines) == 1 and lines[0].endswith("\t%d" % t1) and "512x64*8" in lines[0]
    ens = Ensemble(members, series_capacity=10)
    assert ens.autotune(4, table=table) == t1
    assert len(open(table).read().splitlines()) == 1
    ens.set_collision("central", 1.0, 1.0, 1.0)
    ens.autotune(4, table=table)
    assert len(open(table).read().splitlines()) == 2
    ens.init(1, 1e-3)  # tuned before init, as the call requires
    ens.step(3)
    assert int(ens.flags().sum()) == 0
    ens.close()


def _uneven():
    """Three runs of lattice shapes (an uneven batch), squares across strip and row-range seams."""
    return ([workloads.Member(256, 64, 0.6, 2e-5, (100, 30, 6))] * 3 +
            [workloads.Member(512, 128, 0.57, 1e-5, (250, 60, 8))] * 2 +
            [workloads.Member(1024, 96, 0.55, 1e-5, (510, 30, 8))] * 2)


def test_run_rows_per_lattice_size_bit_identical():
    """Row ranges chosen per run of lattice shapes (whole strips, 64, 32 and 16 rows) in two-step
    launches: every state and drag value equals those of whole strips, for both collisions, over
    an odd number of steps; get_run_rows reports what each run uses; bad arguments change
    nothing."""
    members = _uneven()
    for collision in (None, (1.0, 1.0, 1.0)):
        runs = []
        for rows in (None, [0, 32, 16], [64, 0, 32], [-1, 16, 0]):
            ens = _ensemble(members, 60)
            ens.set_tile(16)  # two steps per launch, whole strips
            if collision is not None:
                ens.set_collision("central", *collision)
            assert ens.run_count() == 3
            if rows is not None:
                ens.set_run_rows(rows)
                expect = [0 if r <= 0 or r >= m.ny else r for r, m in zip(rows, (members[0], members[3], members[5]))]
                assert ens.run_rows() == expect
            else:
                assert ens.run_rows() == [0, 0, 0]
            ens.init(5, 1e-2)
            ens.step(41)
            torch.cuda.synchronize()
            runs.append((ens.drag(0, 42).cpu().numpy(), [ens.state(i).cpu().numpy().copy() for i in (0, 3, 4, 6)]))
            ens.close()
        d0, s0 = runs[0]
        for d, st in runs[1:]:
            assert np.array_equal(d, d0), collision
            for i, (a, b) in zip((0, 3, 4, 6), zip(st, s0)):
                fluid = ~olbm.solid_mask(_channel(members[i]))
                assert np.array_equal(a[:, fluid], b[:, fluid]), (collision, i)
    ens = _ensemble(members, 10)
    ens.set_tile(16)
    ens.set_run_rows([0, 32, 16])
    for bad in ([0, 32], [0, 32, 16, 8], [0, -2, 16]):
        with pytest.raises(RuntimeError):
            ens.set_run_rows(bad)
        assert ens.run_rows() == [0, 32, 16]
    ens.set_run_rows(None)
    assert ens.run_rows() == [0, 0, 0]
    ens.set_tile(0)
    assert ens.run_rows() == [-1, -1, -1]
    ens.close()


def test_autotune_per_lattice_size(tmp_path):
    """On an uneven batch the tuner keeps one row range per run when it is clearly faster; the
    table line carries them, a new context reads them back, and the tuned ensemble steps to the
    same states as the default shape."""
    from paper_2005_09323_amd.ensemble import Ensemble
    members = _uneven()
    table = str(tmp_path / "tiles.txt")
    ens = Ensemble(members, series_capacity=40)
    tile = ens.autotune(4, table=table)
    rows = ens.run_rows()
    assert len(rows) == 3
    line = open(table).read().splitlines()[0]
    key, val = line.split("\t")
    assert "256x64*3;512x128*2;1024x96*2;" in key
    if ens.launch_steps() == 2 and ens.run_rows()[0] != -1:
        assert val.split()[0] == str(tile) and len(val.split()) == 2
        assert [int(v) for v in val.split()[1].split(",")] == rows
    ens.init(2, 1e-2)
    ens.step(33)
    torch.cuda.synchronize()
    tuned = [ens.state(i).cpu().numpy().copy() for i in (0, 3, 6)]
    d_tuned = ens.drag(0, 34).cpu().numpy()
    ens.close()
    ens = Ensemble(members, series_capacity=40)
    assert ens.autotune(4, table=table) == tile
    assert ens.run_rows() == rows
    ens.close()
    ens = Ensemble(members, series_capacity=40)
    ens.set_tile(0)
    ens.init(2, 1e-2)
    ens.step(33)
    torch.cuda.synchronize()
    assert np.array_equal(ens.drag(0, 34).cpu().numpy(), d_tuned)
    for i, a in zip((0, 3, 6), tuned):
        fluid = ~olbm.solid_mask(_channel(members[i]))
        assert np.array_equal(ens.state(i).cpu().numpy()[:, fluid], a[:, fluid]), i
    ens.close()


def test_adaptive_shape_cuts_strips_for_a_mid_sized_batch():
    """32 members of 1024 x 256 give 128 whole strips, too few for the device: the default shape
    cuts them into row ranges and still makes two steps per launch; 8 of them active fall back to
    one step.  Every state and drag value equals those of the one-step shape 0."""
    m = workloads.Member(1024, 256, 0.51, 2e-6, (240, 112, 32))
    runs = []
    for tile in (None, 0):
        ens = _ensemble([m] * 32, 80)
        if tile is not None:
            ens.set_tile(tile)
        ens.init(3, 1e-3)
        if tile is None:
            assert ens.launch_steps() == 2
        ens.step(37)
        ens.set_active([1] * 8 + [0] * 24)
        if tile is None:
            assert ens.launch_steps() == 1
        ens.step(5)
        ens.set_active(None)
        ens.step(30)
        torch.cuda.synchronize()
        runs.append(([ens.time(i) for i in (0, 8)], ens.drag(0, 73).cpu().numpy(),
                     [ens.state(i).cpu().numpy().copy() for i in (0, 13, 31)]))
        ens.close()
        torch.cuda.empty_cache()
    (t0, d0, s0), (t1, d1, s1) = runs
    assert t0 == t1 == [73, 68]
    assert np.array_equal(d0[:8], d1[:8]) and np.array_equal(d0[8:, :68], d1[8:, :68])
    fluid = ~olbm.solid_mask(_channel(m))
    for a, b in zip(s0, s1):
        assert np.array_equal(a[:, fluid], b[:, fluid])
