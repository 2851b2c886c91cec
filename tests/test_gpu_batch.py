"""GPU: batches of uneven channels (lbm_batch_*) against the same channels
stepped alone, and against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2403_15768_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_15768_amd import lbm as mod

    mod.load()
    return mod


def say(*a):
    print(*a, flush=True)


def make_ducts(lbm, specs, precision):
    out = []
    for k, (nx, ny, nz, tau, g) in enumerate(specs):
        ch = lbm.Channel(19, lbm.DUCT, nx, ny, nz, tau=tau, force=(g, 0, 0), precision=precision)
        ch.set_friction(inputs.duct_friction(ch.wall_coords(), nx, ny, nz, inputs.rng_for("batch", 100 + k),
                                             sigma=6.0))
        out.append(ch)
    return out


SPECS = [(37, 12, 9, 0.65, 2e-6), (64, 10, 14, 0.9, 1e-6), (100, 8, 8, 1.1, 1.5e-6),
         (128, 16, 12, 0.7, 0.7e-6), (33, 9, 11, 0.6, 1.2e-6)]


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s"])
def test_batch_bit_identical_to_alone(lbm, precision):
    say("batch vs alone", precision)
    alone = make_ducts(lbm, SPECS, precision)
    mixed = make_ducts(lbm, SPECS, precision)
    for ch in alone:
        ch.step(20)
    for ch in mixed:
        ch.step(20)  # members join with some history (different parities)
    mixed[1].step(1)
    alone[1].step(1)
    b = lbm.Batch(mixed)
    b.step(150)  # 2 graph replays + 22 single launches
    for ch in alone:
        ch.step(150)
    for a, m in zip(alone, mixed):
        assert m.step_count == a.step_count
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    inv_b = b.invariants()
    for k, a in enumerate(alone):
        q, mass, dm = a.invariants()
        assert abs(inv_b[k, 0] / q - 1) < 1e-13
        assert abs(inv_b[k, 1] - mass) < 1e-9
    b.close()


@pytest.mark.parametrize("shape", [1, 2, 8])
def test_half_storage_batch_shapes_bit_identical(lbm, shape):
    # the half-storage kernel takes the plain items two to a wave (with one
    # wave per workgroup a pair spans two workgroups, and an odd count leaves
    # one item alone); the other shapes besides the default, over a graph
    # replay and an odd number of single launches
    say("half-storage batch, waves per workgroup", shape)
    alone = make_ducts(lbm, SPECS, "f16s")
    mixed = make_ducts(lbm, SPECS, "f16s")
    b = lbm.Batch(mixed)
    b.set_shape(shape)
    b.step(67)
    for ch in alone:
        ch.step(67)
    for a, m in zip(alone, mixed):
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    b.close()


TUBES = ((6, 40, 0), (9, 70, 1), (4, 64, 2))  # radius, nx, seed


def tube_spectral(seed):
    return inputs.draw_spectral(inputs.rng_for("serving", 10 + seed), nq=16, nw=64)


def tube_omega(coords, nx, R, cy, cz, sp, seed):
    return inputs.tube_plasmon_frequencies(coords, nx, R, cy, cz, sp.omega0,
                                           inputs.rng_for("serving", 20 + seed), sigma=4.0)


@pytest.mark.parametrize("precision", ["f16s", "f32", "f64"])
def test_batch_tubes_bit_identical(lbm, precision):
    # tubes (interpolated bounce-back) in a batch: the batch kernel's BOUZ
    # path against the channel kernel, bit for bit, in every storage
    say("batch tubes", precision)
    chans = []
    for R, nx, seed in TUBES:
        ny, nz, cy, cz = inputs.tube_box(R)
        pair = []
        for _ in range(2):
            ch = lbm.Channel(19, lbm.TUBE, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0),
                             precision=precision, tube_radius=float(R), tube_cy=cy, tube_cz=cz)
            sp = tube_spectral(seed)
            ch.set_friction_spectral(sp, tube_omega(ch.wall_coords(), nx, R, cy, cz, sp, seed))
            pair.append(ch)
        chans.append(pair)
    for p in chans:  # join the batch at an odd step
        p[0].step(3)
        p[1].step(3)
    b = lbm.Batch([p[1] for p in chans])
    b.step(100)
    for p in chans:
        p[0].step(100)
        assert p[0].step_count == p[1].step_count == 103
        assert np.array_equal(p[0].get_state()[0], p[1].get_state()[0])
    b.close()


def test_batch_tubes_fp64_against_oracle(lbm):
    # the batched tubes against the oracle, friction from the oracle's own
    # quadrature of the same spectra
    say("batch tubes fp64 vs oracle")
    chans, oras = [], []
    for R, nx, seed in TUBES:
        ny, nz, cy, cz = inputs.tube_box(R)
        kw = dict(tube_radius=float(R), tube_cy=cy, tube_cz=cz)
        ch = lbm.Channel(19, lbm.TUBE, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0), precision="f64",
                         **kw)
        sp = tube_spectral(seed)
        om = tube_omega(ch.wall_coords(), nx, R, cy, cz, sp, seed)
        ch.set_friction_spectral(sp, om)
        o = oracle.Lattice(19, oracle.TUBE, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0), **kw)
        _, lam = oracle.friction(oracle.Spectral(T=sp.T, omega0=sp.omega0, gamma_s=sp.gamma_s,
                                                 omega_l=sp.omega_l, gamma_l=sp.gamma_l,
                                                 a_l=sp.a_l, d=sp.d, nq=sp.nq, nw=sp.nw,
                                                 lambda_target=sp.lambda_target), om)
        o.set_friction(lam)
        chans.append(ch)
        oras.append(o)
    b = lbm.Batch(chans)
    b.step(300)
    for ch, o in zip(chans, oras):
        o.step(300)
        ug, uo = ch.field(1), o.fields()[1]
        err = np.max(np.abs(ug - uo)) / np.max(np.abs(uo))
        say("  err", err)
        assert err < 1e-12
    b.close()


def test_batch_fp64_against_oracle(lbm):
    say("batch fp64 vs oracle")
    specs = SPECS[:3]
    chans = make_ducts(lbm, specs, "f64")
    b = lbm.Batch(chans)
    b.step(300)
    for k, (nx, ny, nz, tau, g) in enumerate(specs):
        o = oracle.Lattice(19, oracle.DUCT, nx, ny, nz, tau=tau, force=(g, 0, 0))
        o.set_friction(inputs.duct_friction(o.wall_coords(), nx, ny, nz, inputs.rng_for("batch", 100 + k),
                                            sigma=6.0))
        o.step(300)
        ug, uo = chans[k].field(1), o.fields()[1]
        err = np.max(np.abs(ug - uo)) / np.max(np.abs(uo))
        say("  member", k, "err", err)
        assert err < 1e-12


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_slab_and_duct_members(lbm, precision):
    """Planar members of both kinds in one batch: D3Q19 slabs (z periodic, so
    the columns at the z boundary take the general path) beside ducts, bit-
    identical to the same channels alone, and the FP64 slab against the oracle."""
    say("batch slab + duct", precision)
    shapes = [(lbm.SLAB, 40, 9, 6, 0.75), (lbm.DUCT, 37, 10, 8, 0.9), (lbm.SLAB, 100, 7, 3, 0.6),
              (lbm.SLAB, 64, 12, 1, 0.8)]

    def make():
        out = []
        for k, (geom, nx, ny, nz, tau) in enumerate(shapes):
            ch = lbm.Channel(19, geom, nx, ny, nz, tau=tau, force=(1e-6, 0, 0), precision=precision)
            lam = inputs.duct_friction(ch.wall_coords(), nx, ny, nz, inputs.rng_for("batch", 300 + k),
                                       sigma=4.0)
            ch.set_friction(lam)
            out.append((ch, lam))
        return out

    alone, mixed = make(), make()
    b = lbm.Batch([c for c, _ in mixed])
    b.step(64 + 13)
    for (a, _), (m, _) in zip(alone, mixed):
        a.step(77)
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    if precision == "f64":
        geom, nx, ny, nz, tau = shapes[0]
        o = oracle.Lattice(19, oracle.SLAB, nx, ny, nz, tau=tau, force=(1e-6, 0, 0))
        o.set_friction(mixed[0][1])
        o.step(77)
        ug, uo = mixed[0][0].field(1), o.fields()[1]
        assert np.max(np.abs(ug - uo)) / np.max(np.abs(uo)) < 1e-12
    b.close()


def test_batch_tune_leaves_state(lbm):
    say("batch tune")
    chans = make_ducts(lbm, SPECS, "f32")
    b = lbm.Batch(chans)
    b.step(10)
    before = [c.get_state()[0].copy() for c in chans]
    w = b.tune()
    assert w in (1, 2, 4, 8)
    for c, s in zip(chans, before):
        assert np.array_equal(c.get_state()[0], s) and c.step_count == 10
    ref = make_ducts(lbm, SPECS, "f32")
    for c in ref:
        c.step(80)
    b.step(70)
    for c, r in zip(chans, ref):
        assert np.array_equal(c.get_state()[0], r.get_state()[0])


def test_batch_members_stepped_outside(lbm):
    """Members advanced or restored on their own between batch steps: the
    batch picks up their current step and buffer, and stays bit-identical."""
    say("batch with members stepped outside")
    chans = make_ducts(lbm, SPECS, "f16s")
    ref = make_ducts(lbm, SPECS, "f16s")
    b = lbm.Batch(chans)
    b.step(70)
    chans[0].step(3)   # odd: parity flips
    chans[2].step(64)  # through the channel's own graph
    b.step(65)
    saved = chans[3].get_state()
    b.step(5)
    chans[3].set_state(*saved)  # back 5 steps
    b.step(5)
    inv_b = b.invariants()
    plan = [148, 145, 209, 140, 145]
    for k, (c, r) in enumerate(zip(chans, ref)):
        r.step(plan[k])
        assert c.step_count == r.step_count == plan[k]
        assert np.array_equal(c.get_state()[0], r.get_state()[0])
        q, mass, dm = r.invariants()
        assert abs(inv_b[k, 0] / q - 1) < 1e-13
    b.close()


@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_batch_groups_do_not_change_results(lbm, precision):
    """Members cut into several groups (each run 64 steps before the next)
    give the same bits as one group stepped in lockstep, and as alone."""
    say("batch groups", precision)
    one = make_ducts(lbm, SPECS, precision)
    many = make_ducts(lbm, SPECS, precision)
    alone = make_ducts(lbm, SPECS, precision)
    b1 = lbm.Batch(one)
    b1.set_group_bytes(0)
    assert b1.groups == 1
    bn = lbm.Batch(many)
    bn.set_group_bytes(1)  # every member its own group
    assert bn.groups == len(SPECS)
    for b in (b1, bn):
        b.step(64 * 3 + 7)
        b.step(5)
    for c in alone:
        c.step(204)
    for a, x, y in zip(alone, one, many):
        ref = a.get_state()[0]
        assert np.array_equal(x.get_state()[0], ref)
        assert np.array_equal(y.get_state()[0], ref)
    i1, i2 = b1.invariants(), bn.invariants()
    assert np.array_equal(i1, i2)
    bn.set_group_bytes(3 * many[0].get_state()[0].nbytes)  # regroup mid-run
    bn.set_streams(3)
    b1.set_streams(1)
    bn.step(70)
    b1.step(70)
    for x, y in zip(one, many):
        assert np.array_equal(x.get_state()[0], y.get_state()[0])
    b1.close()
    bn.close()


def test_batch_full_size_sampled(lbm):
    """The 256-duct batch at full size (48 M cells), in the configuration the
    benchmark times (default groups and streams): sampled members are bit-
    identical to the same channels stepped alone, and the smallest one agrees
    with the oracle (FP64 run of the same member)."""
    say("batch full size")
    specs = inputs.batch_channels(256)
    chans = []
    for k, c in enumerate(specs):
        ch = lbm.Channel(19, lbm.DUCT, c.nx, c.ny, c.nz, tau=c.tau, force=(c.g, 0, 0), precision="f32")
        ch.set_friction(inputs.duct_friction(ch.wall_coords(), c.nx, c.ny, c.nz,
                                             inputs.rng_for("batch", c.seed_index)))
        chans.append(ch)
    b = lbm.Batch(chans)
    assert b.groups > 1
    b.step(64 + 9)
    inv = b.invariants()
    small = min(range(len(specs)), key=lambda k: specs[k].nx * specs[k].ny * specs[k].nz)
    for k in sorted({0, 101, 255, small}):
        c = specs[k]
        a = lbm.Channel(19, lbm.DUCT, c.nx, c.ny, c.nz, tau=c.tau, force=(c.g, 0, 0), precision="f32")
        a.set_friction(inputs.duct_friction(a.wall_coords(), c.nx, c.ny, c.nz,
                                            inputs.rng_for("batch", c.seed_index)))
        a.step(73)
        assert np.array_equal(a.get_state()[0], chans[k].get_state()[0]), k
        assert abs(inv[k, 0] / a.invariants()[0] - 1) < 1e-13
        a.close()
    c = specs[small]
    o = oracle.Lattice(19, oracle.DUCT, c.nx, c.ny, c.nz, tau=c.tau, force=(c.g, 0, 0))
    o.set_friction(inputs.duct_friction(o.wall_coords(), c.nx, c.ny, c.nz,
                                        inputs.rng_for("batch", c.seed_index)))
    o.step(73)
    ug, uo = chans[small].field(1), o.fields()[1]
    err = np.max(np.abs(ug - uo)) / np.max(np.abs(uo))
    say("  smallest member vs oracle", err)
    assert err < 1e-5
    b.close()
    for ch in chans:
        ch.close()


def test_batch_rejects_bad_settings(lbm):
    chans = make_ducts(lbm, SPECS[:2], "f32")
    b = lbm.Batch(chans)
    for bad in (0, 3, 16):
        with pytest.raises(lbm.LBMError):
            b.set_shape(bad)
    for bad in (0, 5):
        with pytest.raises(lbm.LBMError):
            b.set_streams(bad)
    with pytest.raises(lbm.LBMError):
        b.step(-1)
    b.set_shape(8)
    b.set_streams(4)
    b.step(3)  # still usable
    assert all(c.step_count == 3 for c in chans)
    b.close()


def test_batch_rejects_mixed_members(lbm):
    a = lbm.Channel(19, lbm.DUCT, 16, 6, 6, tau=0.7, precision="f32")
    c = lbm.Channel(19, lbm.DUCT, 16, 6, 6, tau=0.7, precision="f64")
    with pytest.raises(lbm.LBMError):
        lbm.Batch([a, c])
    with pytest.raises(lbm.LBMError):
        lbm.Batch([a, a])


# ---------------------------------------------- members joining and leaving
def capacity_for(lbm, chans, members=None, slack=1):
    items = cols = 0
    for ch in chans:
        i, c = lbm.member_cost(ch)
        items, cols = items + i, cols + c
    return dict(max_members=members or len(chans), max_items=slack * items,
                max_columns=slack * cols)


@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_members_join_and_leave_bit_identical_to_alone(lbm, precision):
    # members join a running batch at different steps and leave again; each
    # is bit for bit the channel stepped alone the same number of steps, and
    # the batch's reductions match each member's own
    say("batch add / remove", precision)
    alone = make_ducts(lbm, SPECS, precision)
    mixed = make_ducts(lbm, SPECS, precision)
    cap = capacity_for(lbm, mixed, members=4, slack=2)
    b = lbm.Batch.empty(19, precision, False, **cap)
    steps = [0] * len(SPECS)

    def run(n, active):
        b.step(n)
        for k in active:
            steps[k] += n

    assert b.add(mixed[0]) == 0
    assert b.add(mixed[1]) == 1
    run(70, [0, 1])
    mixed[2].step(5)  # joins with a history (another buffer parity)
    steps[2] += 5
    assert b.add(mixed[2]) == 2
    run(64, [0, 1, 2])
    b.remove(mixed[1])  # leaves from the middle: its slot is free again
    assert b.members == 2 and b.channels[1] is None
    assert b.add(mixed[3]) == 1
    assert b.add(mixed[4]) == 3
    with pytest.raises(lbm.LBMError):
        b.add(mixed[1])  # four slots, all taken
    run(131, [0, 2, 3, 4])
    inv = b.invariants()
    for k, slot in ((0, 0), (2, 2), (3, 1), (4, 3)):
        assert abs(inv[slot, 0] / mixed[k].invariants()[0] - 1) < 1e-13
    b.remove(mixed[0])
    mixed[1].step(3)  # stepped alone meanwhile, then back in
    steps[1] += 3
    assert b.add(mixed[1]) == 0
    run(64, [1, 2, 3, 4])
    for a, m, n in zip(alone, mixed, steps):
        a.step(n)
        assert m.step_count == a.step_count == n
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    with pytest.raises(lbm.LBMError):
        b.remove(mixed[0])  # not a member any more
    with pytest.raises(lbm.LBMError):
        b.add(mixed[2])  # a member already
    b.close()


def test_join_and_leave_across_groups_and_repacks(lbm):
    # small groups (one member each) and a work list with little room: joins
    # and leaves move groups to fresh regions and repack the list; results
    # stay bit for bit those of the channels alone
    say("batch groups + repack")
    specs = SPECS * 2
    alone = make_ducts(lbm, specs, "f32")
    mixed = make_ducts(lbm, specs, "f32")
    cap = capacity_for(lbm, mixed)
    b = lbm.Batch.empty(19, "f32", False, **cap)
    b.set_group_bytes(2 * mixed[0].get_state()[0].nbytes + 1)
    for ch in mixed[:6]:
        b.add(ch)
    b.step(64)
    for k in (1, 4):
        b.remove(mixed[k])
    for ch in mixed[6:]:
        b.add(ch)
    b.step(65)
    b.add(mixed[1])
    b.step(64)
    assert b.settings()["repacks"] >= 1
    n = {0: 193, 2: 193, 3: 193, 5: 193, 4: 64, 1: 128, 6: 129, 7: 129, 8: 129, 9: 129}
    for k, (a, m) in enumerate(zip(alone, mixed)):
        a.step(n[k])
        assert np.array_equal(a.get_state()[0], m.get_state()[0]), k
    b.close()


def test_tuning_is_cached_and_never_changes_results(lbm):
    say("batch autotuner")
    alone = make_ducts(lbm, SPECS, "f32")
    mixed = make_ducts(lbm, SPECS, "f32")
    b = lbm.Batch(mixed)
    b.tune(retime=True)
    t = b.tuning
    assert t["waves_per_group"] in (2, 4, 8) and t["streams"] in (1, 2, 3)
    assert t["us_per_step"] > 0 and t["us_per_step"] <= t["us_per_step_default"] * 1.05
    assert t["cached"] == 0
    b.step(100)
    for a in alone:
        a.step(100)
    for a, m in zip(alone, mixed):
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    # the same kind and size of batch: the cached choice, no timing
    again = make_ducts(lbm, SPECS, "f32")
    b2 = lbm.Batch(again)
    b2.tune()
    assert b2.tuning["cached"] == 1
    s = b2.settings()
    assert (s["waves_per_group"], s["group_bytes"], s["streams"]) == \
        (t["waves_per_group"], t["group_bytes"], t["streams"])
    b.close()
    b2.close()


# ---------------------------------------------------------- open x ends
# members with open ends (each its own end densities) step bit for bit as
# alone: the batch kernel takes the ghosts from each member's end-node records
OPEN_SPECS = SPECS + [(150, 9, 7, 0.8, 1e-6)]  # and one padded x-line


def open_ducts(lbm, precision):
    chans = make_ducts(lbm, OPEN_SPECS, precision)
    for k, ch in enumerate(chans):
        ch.set_open_ends(1.0 + 1e-5 * (k + 1), 1.0 - 0.7e-5 * (k + 1))
    return chans


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_open_end_batch_bit_identical_to_alone(lbm, precision):
    say("open batch vs alone", precision)
    alone = open_ducts(lbm, precision)
    mixed = open_ducts(lbm, precision)
    for ch in alone + mixed:
        ch.step(20)
    alone[2].step(1)
    mixed[2].step(1)
    b = lbm.Batch(mixed)
    b.step(150)
    for ch in alone:
        ch.step(150)
    for a, m in zip(alone, mixed):
        assert m.step_count == a.step_count
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    inv = b.invariants()
    for k, a in enumerate(alone):
        q, mass, _ = a.invariants()
        assert abs(inv[k, 0] / q - 1) < 1e-13
        assert abs(inv[k, 1] / mass - 1) < 1e-14
    b.close()


@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_open_end_tube_batch_bit_identical_to_alone(lbm, precision):
    say("open tube batch vs alone", precision)

    def tubes():
        out = []
        for k, (R, nx, seed) in enumerate(TUBES):
            n = int(2 * R + 4)
            c = (n - 1) / 2
            t = lbm.Channel(19, lbm.TUBE, nx, n, n, tau=0.8, force=(1e-6, 0, 0),
                            precision=precision, tube_radius=float(R), tube_cy=c, tube_cz=c)
            t.set_friction(np.random.default_rng(seed).uniform(0.0, 0.3, t.wall_count))
            t.set_open_ends(1.0 + 2e-5, 1.0 - 1e-5 * (k + 1))
            out.append(t)
        return out

    alone, mixed = tubes(), tubes()
    b = lbm.Batch(mixed)
    b.step(137)
    for a, m in zip(alone, mixed):
        a.step(137)
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    b.close()


def test_open_end_batch_fp64_against_oracle(lbm):
    say("open batch vs oracle")
    chans = open_ducts(lbm, "f64")
    b = lbm.Batch(chans)
    b.step(229)
    for k in (0, 3, 5):
        nx, ny, nz, tau, g = OPEN_SPECS[k]
        o = oracle.Lattice(19, oracle.DUCT, nx, ny, nz, tau=tau, force=(g, 0, 0))
        o.set_friction(inputs.duct_friction(o.wall_coords(), nx, ny, nz,
                                            inputs.rng_for("batch", 100 + k), sigma=6.0))
        o.set_open_ends(1.0 + 1e-5 * (k + 1), 1.0 - 0.7e-5 * (k + 1))
        o.step(229)
        ug, uo = chans[k].field(1), o.fields()[1]
        err = np.max(np.abs(ug - uo)) / np.max(np.abs(uo))
        say(f"  member {k}: {err:.2e}")
        assert err < 1e-12
    b.close()


def test_open_end_members_join_leave_and_change_densities(lbm):
    # open-ended members join a running batch, one changes its end densities
    # between batch steps, one leaves and steps alone: bit for bit the
    # channels stepped alone; periodic channels are refused
    say("open batch add / remove")
    alone = open_ducts(lbm, "f32")
    mixed = open_ducts(lbm, "f32")
    cap = capacity_for(lbm, mixed, members=4, slack=2)
    b = lbm.Batch.empty(19, "f32", False, open_ends=True, **cap)
    periodic = make_ducts(lbm, SPECS[:1], "f32")[0]
    with pytest.raises(lbm.LBMError):
        b.add(periodic)
    for k in (0, 1, 5):
        b.add(mixed[k])
    b.step(70)
    for k in (0, 1, 5):
        alone[k].step(70)
    for ch in (mixed[1], alone[1]):
        ch.set_open_ends(1.0 + 4e-5, 1.0 - 1e-5)
    b.step(64)
    for k in (0, 1, 5):
        alone[k].step(64)
    b.remove(mixed[0])
    mixed[0].step(9)
    alone[0].step(9)
    b.add(mixed[0])
    b.add(mixed[3])
    b.step(131)
    for k in (0, 1, 3, 5):
        alone[k].step(131)
    for k in (0, 1, 3, 5):
        assert np.array_equal(alone[k].get_state()[0], mixed[k].get_state()[0]), k
    b.close()


# ------------------------------------------------------------ electron lines
# members with electron lines (each its own line parameters, some with
# phonon lines): a batch step runs each group's line step, then its water
# step, bit for bit as the channels alone
ELEC_SPECS = [(37, 12, 9, 0.65, 2e-6, "duct"), (64, 10, 14, 0.9, 1e-6, "slab"),
              (100, 8, 8, 1.1, 1.5e-6, "duct"), (33, 9, 11, 0.6, 1.2e-6, "slab"),
              (150, 9, 7, 0.8, 1e-6, "duct")]


def electron_channels(lbm, precision):
    out = []
    for k, (nx, ny, nz, tau, g, geom) in enumerate(ELEC_SPECS):
        ch = lbm.Channel(19, lbm.DUCT if geom == "duct" else lbm.SLAB, nx, ny, nz, tau=tau,
                         force=(g, 0, 0), precision=precision)
        ch.set_friction(np.random.default_rng(40 + k).uniform(0.0, 0.3, ch.wall_count))
        ch.set_electrons(0.8 + 0.05 * k, 0.7 + 0.2 * k, 0.03, -1e-6 * (k - 2))
        if k % 2:
            ch.set_phonons(0.7, 1.3, 0.02, 0.08)
        out.append(ch)
    return out


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_electron_batch_bit_identical_to_alone(lbm, precision):
    say("electron batch vs alone", precision)
    alone = electron_channels(lbm, precision)
    mixed = electron_channels(lbm, precision)
    for ch in alone + mixed:
        ch.step(20)
    alone[1].step(1)
    mixed[1].step(1)
    b = lbm.Batch(mixed)
    b.step(150)
    for ch in alone:
        ch.step(150)
    for a, m in zip(alone, mixed):
        assert m.step_count == a.step_count
        assert np.array_equal(a.get_state()[0], m.get_state()[0])  # water and lines
        assert np.array_equal(a.electrons()[0], m.electrons()[0])
    inv = b.invariants()
    for k, a in enumerate(alone):
        assert abs(inv[k, 0] / a.invariants()[0] - 1) < 1e-13
    b.close()


def test_electron_tube_batch_bit_identical_to_alone(lbm):
    say("electron tube batch vs alone")

    def tubes():
        out = []
        for k, (R, nx, seed) in enumerate(TUBES):
            n = int(2 * R + 4)
            c = (n - 1) / 2
            t = lbm.Channel(19, lbm.TUBE, nx, n, n, tau=0.8, force=(1e-6, 0, 0),
                            precision="f32", tube_radius=float(R), tube_cy=c, tube_cz=c)
            t.set_friction(np.random.default_rng(seed).uniform(0.0, 0.3, t.wall_count))
            t.set_electrons(0.85, 0.9 + 0.3 * k, 0.05, 2e-6)
            out.append(t)
        return out

    alone, mixed = tubes(), tubes()
    b = lbm.Batch(mixed)
    b.step(137)
    for a, m in zip(alone, mixed):
        a.step(137)
        assert np.array_equal(a.get_state()[0], m.get_state()[0])
    b.close()


def test_electron_batch_fp64_against_oracle(lbm):
    say("electron batch vs oracle")
    chans = electron_channels(lbm, "f64")
    b = lbm.Batch(chans)
    b.step(101)
    for k in (0, 1):
        nx, ny, nz, tau, g, geom = ELEC_SPECS[k]
        o = oracle.Lattice(19, oracle.DUCT if geom == "duct" else oracle.SLAB, nx, ny, nz,
                           tau=tau, force=(g, 0, 0))
        o.set_friction(np.random.default_rng(40 + k).uniform(0.0, 0.3, o.wall_count))
        o.set_electrons(0.8 + 0.05 * k, 0.7 + 0.2 * k, 0.03, -1e-6 * (k - 2))
        if k % 2:
            o.set_phonons(0.7, 1.3, 0.02, 0.08)
        o.step(101)
        ug, uo = chans[k].field(1), o.fields()[1]
        err = np.max(np.abs(ug - uo)) / np.max(np.abs(uo))
        eg, eo = chans[k].electrons()[0], o.electrons()[0]
        eerr = np.abs(eg - eo).max() / np.abs(eo).max()
        say(f"  member {k}: water {err:.2e} u_e {eerr:.2e}")
        assert err < 1e-12 and eerr < 1e-12
    b.close()


def test_electron_members_join_leave_and_change(lbm):
    say("electron batch add / remove")
    alone = electron_channels(lbm, "f32")
    mixed = electron_channels(lbm, "f32")
    cap = capacity_for(lbm, mixed, members=3, slack=2)
    b = lbm.Batch.empty(19, "f32", False, electrons=True, **cap)
    plain = make_ducts(lbm, SPECS[:1], "f32")[0]
    with pytest.raises(lbm.LBMError):
        b.add(plain)  # no electron lines
    for k in (0, 2, 3):
        b.add(mixed[k])
    b.step(70)
    for k in (0, 2, 3):
        alone[k].step(70)
    for ch in (mixed[2], alone[2]):  # new line parameters (lines reset to rest)
        ch.set_electrons(0.9, 1.1, 0.01, 3e-6)
    b.step(64)
    for k in (0, 2, 3):
        alone[k].step(64)
    b.remove(mixed[0])
    b.add(mixed[4])
    b.step(65)
    for k in (2, 3, 4):
        alone[k].step(65)
    for k in (0, 2, 3, 4):
        assert np.array_equal(alone[k].get_state()[0], mixed[k].get_state()[0]), k
    b.close()
