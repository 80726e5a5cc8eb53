"""Batched form: uneven lattices advanced by one fused pass per stage and a
captured graph are bit-identical to the same lattices advanced alone, across
graph replays with eager work in between, membership changes and both
storage precisions."""
import numpy as np
import pytest

import paper_1201_5029_amd as sl
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


def _runs(precision, sizes, base_seed=20120200):
    rs = []
    for j, n in enumerate(sizes):
        r = synth.preheat(n=n, order=4, dt=0.005, precision=precision, seed=base_seed + j,
                          phi0=1.0 + (j - len(sizes) // 2) * 1e-5)
        rs.append(r)
    return rs


def _same(a, b):
    fa, pa = a.get_fields()
    fb, pb = b.get_fields()
    return np.array_equal(fa, fb) and np.array_equal(pa, pb) and a.background() == b.background()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batched_equals_alone_over_graph_replays(precision):
    sl.symlat.load().sl_autotune_forget()    # members keep their own shapes
    recipes = _runs(precision, [32, 64, 48, 32, 96])
    alone = [sl.from_recipe(r) for r in recipes]
    mixed = [sl.from_recipe(r) for r in recipes]
    for a, m in zip(alone, mixed):
        assert a.tile() == m.tile() and _same(a, m)
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    assert len(b) == len(mixed)
    for rep in range(4):           # the second and later calls replay the graph
        b.step(10, 0.005, 4)
        for a in alone:
            a.evolve(10, 0.005, 4)  # eager launches between replays
        b.synchronize()
        for j, (a, m) in enumerate(zip(alone, mixed)):
            assert _same(a, m), (rep, j, recipes[j]["n"])
    e = mixed[2].energies()
    say(precision, "batched residual", e["friedmann_residual"], "a", e["a"])
    assert e["friedmann_residual"] < (1e-3 if precision == "f32" else 1e-8)


def test_membership_changes_and_mixed_calls():
    sl.symlat.load().sl_autotune_forget()
    recipes = _runs("f32", [32, 64, 96, 64])
    alone = [sl.from_recipe(r) for r in recipes]
    mixed = [sl.from_recipe(r) for r in recipes]
    b = sl.Batch()
    b.add(mixed[0])
    b.add(mixed[1])
    b.step(5, 0.005, 4)
    alone[0].evolve(5, 0.005, 4)
    alone[1].evolve(5, 0.005, 4)
    # a member evolved on its own between batched calls stays ordered
    mixed[1].evolve(3, 0.005, 4)
    alone[1].evolve(3, 0.005, 4)
    b.add(mixed[2])                 # joins late: its own step count
    b.step(7, 0.005, 4)
    for k in (0, 1, 2):
        alone[k].evolve(7, 0.005, 4)
    b.remove(mixed[0])
    b.add(mixed[3])
    b.step(4, 0.005, 4)
    for k in (1, 2, 3):
        alone[k].evolve(4, 0.005, 4)
    for k in range(4):
        assert _same(alone[k], mixed[k]), k
    # destroying a member removes it from the batch
    mixed[2].close()
    assert len(b) == 2
    b.step(2, 0.005, 4)
    alone[1].evolve(2, 0.005, 4)
    alone[3].evolve(2, 0.005, 4)
    assert _same(alone[1], mixed[1]) and _same(alone[3], mixed[3])


def test_batch_rejects_mismatched_members():
    b = sl.Batch()
    a = sl.from_recipe(synth.preheat(n=32, precision="f32"))
    c = sl.from_recipe(synth.preheat(n=32, precision="f64"))
    b.add(a)
    with pytest.raises(sl.SymlatError):
        b.add(c)
    with pytest.raises(sl.SymlatError):
        b.add(a)                     # already a member
    osc = sl.from_recipe(synth.oscillon(n=32))
    with pytest.raises(sl.SymlatError):
        b.add(osc)                   # different potential family
    for bad in (-1, (1 << 24) + 1):
        with pytest.raises(sl.SymlatError):
            b.set_grid(bad)
    assert b.grid() == (0, sum(_tiles(m) for m in b.members))
    for tx in (7, 65):
        with pytest.raises(sl.SymlatError):
            a.set_tile(tx, 1, 0, a.tile()[4])


def test_batch_autotune_keeps_state_and_equals_alone():
    """The batch tuner leaves every member's state untouched, applies its
    shapes to the members, and the batch stays bit-identical to the members
    advanced alone with those shapes; a later member of a tuned size starts
    with the tuned shape."""
    sl.symlat.load().sl_autotune_forget()
    recipes = _runs("f32", [32, 64, 48, 32])
    mixed = [sl.from_recipe(r) for r in recipes]
    before = [m.get_fields() for m in mixed]
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    ms = b.autotune(reps=2)
    say("batch autotune best pass ms", ms, [m.tile() for m in mixed])
    assert ms > 0
    for m, (f0, p0) in zip(mixed, before):
        f1, p1 = m.get_fields()
        assert np.array_equal(f0, f1) and np.array_equal(p0, p1)
    alone = [sl.from_recipe(r) for r in recipes]
    for a, m in zip(alone, mixed):
        tx, vx, _, tz, pf = m.tile()
        a.set_tile(tx, vx, tz, pf)
    b.step(12, 0.005, 4)
    for a in alone:
        a.evolve(12, 0.005, 4)
    b.synchronize()
    for a, m in zip(alone, mixed):
        assert _same(a, m)
    late = sl.from_recipe(_runs("f32", [64], base_seed=20120400)[0])
    b2 = sl.Batch()
    b2.add(late)
    assert late.tile() == mixed[1].tile()
    # a member whose own lane shape differs takes the batch's
    odd = sl.from_recipe(_runs("f32", [40], base_seed=20120500)[0])
    odd.set_tile(16, 1, 0, 1)
    b2.add(odd)
    assert odd.tile()[1] == late.tile()[1] and odd.tile()[4] == late.tile()[4]


def test_history_records_every_step_alone_and_batched():
    """The device history holds (eta, a, p_a, rho) at the end of each step:
    equal bit for bit to the background read after single-step calls,
    through the captured chunks of a long call, and for a batch member."""
    sl.symlat.load().sl_autotune_forget()
    r = _runs("f64", [32])[0]
    ref = sl.from_recipe(r)
    bg = []
    for _ in range(40):
        ref.evolve(1, 0.005, 4)
        bg.append(ref.background())
    one = sl.from_recipe(r)
    one.set_history(100)
    one.evolve(40, 0.005, 4)                      # one captured 32-step chunk + 8 eager
    eta, a, pa, rho = one.history()
    assert len(a) == 40 and np.all(rho > 0)
    assert [tuple(x) for x in zip(eta, a, pa)] == bg
    one.set_history(5)
    one.evolve(10, 0.005, 4)
    assert len(one.history()[0]) == 5             # capacity bound
    mem = sl.from_recipe(r)
    mem.set_history(64)
    b = sl.Batch()
    b.add(mem)
    alone = sl.from_recipe(r)
    tx, vx, _, tz, pf = mem.tile()
    alone.set_tile(tx, vx, tz, pf)
    alone.set_history(64)
    b.step(20, 0.005, 4)
    alone.evolve(20, 0.005, 4)
    b.synchronize()
    hb, ha = mem.history(), alone.history()
    assert all(np.array_equal(x, y) for x, y in zip(hb, ha)) and len(hb[0]) == 20
    phi, pi = mem.get_fields()
    mem.set_fields(phi, pi)                       # a reset restarts the record
    assert len(mem.history()[0]) == 0


def test_member_autotune_keeps_the_batch_lane_shape():
    """Tuning one member alone keeps its per-lane shape (vx, pf), which the
    batch's kernel is built for; the batch then advances it bit for bit
    like the same lattice alone with the tuned shape."""
    sl.symlat.load().sl_autotune_forget()
    recipes = _runs("f32", [32, 64])
    mixed = [sl.from_recipe(r) for r in recipes]
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    alone = sl.from_recipe(recipes[1])
    tx, vx, _, tz, pf = mixed[1].tile()
    alone.set_tile(tx, vx, tz, pf)
    b.step(3, 0.005, 4)
    alone.evolve(3, 0.005, 4)
    mixed[1].autotune(reps=1)
    tx, vx2, _, tz, pf2 = mixed[1].tile()
    assert (vx2, pf2) == (vx, pf)
    alone.set_tile(tx, vx, tz, pf)
    b.step(7, 0.005, 4)
    alone.evolve(7, 0.005, 4)
    b.synchronize()
    assert _same(alone, mixed[1])
    sl.symlat.load().sl_autotune_forget()


def test_batch_synchronize_reports_a_nonfinite_member():
    """A NaN planted in one member's state surfaces as SL_E_NONFINITE at the
    batch's next synchronisation (one gathered read-back of every member's
    scalars), while the finite members keep stepping and report their a."""
    sl.symlat.load().sl_autotune_forget()
    recipes = _runs("f64", [16, 24, 16])
    mixed = [sl.from_recipe(r) for r in recipes]
    phi, pi = mixed[1].get_fields()
    phi[0, 3, 4, 5] = np.nan
    eta, a, p_a = mixed[1].background()
    mixed[1].set_fields(phi, pi, a, p_a)       # explicit p_a: no constraint solve
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    b.step(3, 0.005, 4)
    with pytest.raises(sl.SymlatError) as e:
        b.synchronize()
    assert e.value.status == 5
    for j in (0, 2):
        assert mixed[j].background()[1] > 1.0
    b.remove(mixed[1])
    b.step(2, 0.005, 4)
    b.synchronize()                            # the finite members alone: no error


@pytest.mark.parametrize("grid", [0, 1, 3, 7, 8, 13, 64, 1 << 20])
def test_grid_forms_equal_alone(grid):
    """One workgroup per tile (grid 0) and the persistent form with any
    number of workgroups (fewer than the 8 XCDs, a few per XCD, more than the
    tiles) give the members' alone results bit for bit, over graph replays."""
    sl.symlat.load().sl_autotune_forget()
    recipes = _runs("f32", [32, 64, 48, 96])
    alone = [sl.from_recipe(r) for r in recipes]
    mixed = [sl.from_recipe(r) for r in recipes]
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    b.set_grid(grid)
    tiles = sum(_tiles(m) for m in mixed)
    req, launched = b.grid()
    say("grid", grid, "tiles", tiles, "->", (req, launched))
    assert req == grid and launched == (min(grid, tiles) if grid > 0 else tiles)
    for rep in range(3):            # 10 steps: one captured 8-step chunk + 2 eager
        b.step(10, 0.005, 4)
        for a in alone:
            a.evolve(10, 0.005, 4)
        b.synchronize()
        for j, (a, m) in enumerate(zip(alone, mixed)):
            assert _same(a, m), (grid, rep, j)


def _tiles(lat):
    """Tiles of a lattice's fused pass from its shape (tx, vx, ty, tz, pf)."""
    tx, vx, ty, tz, _ = lat.tile()
    n = lat.n
    return (-(-n // (tx * vx))) * (-(-n // ty)) * (-(-n // tz))


def test_batch_with_fewer_tiles_than_xcds():
    """Batches whose whole tile list is shorter than the number of XCDs
    (one 8^3 lattice in one tile; two 6^3 lattices) advance every tile:
    bit-identical to the lattices alone."""
    sl.symlat.load().sl_autotune_forget()
    for sizes in ([8], [6, 6], [4, 8, 4]):
        recipes = _runs("f64", sizes, base_seed=20120600)
        alone = [sl.from_recipe(r) for r in recipes]
        mixed = [sl.from_recipe(r) for r in recipes]
        b = sl.Batch()
        for m in mixed:
            b.add(m)
        for a, m in zip(alone, mixed):
            _, vx, _, _, pf = m.tile()
            for lat in (m, a):
                lat.set_tile(16, vx, lat.n, pf)   # the whole lattice in one tile
        start = [m.get_fields()[0] for m in mixed]
        tiles = sum(_tiles(m) for m in mixed)
        say("sizes", sizes, "tiles", tiles, "grid", b.grid())
        assert tiles == len(sizes) and b.grid() == (0, tiles)
        b.step(5, 0.005, 4)
        for a in alone:
            a.evolve(5, 0.005, 4)
        b.synchronize()
        for a, m, f0 in zip(alone, mixed, start):
            assert _same(a, m), sizes
            assert not np.array_equal(f0, m.get_fields()[0])   # every lattice moved
        b.close()


def test_member_parameter_change_equals_alone():
    """A batch member given new parameters of its family keeps its tile and
    steps with the new parameters, like the same lattice alone; another
    family is refused while it is a member."""
    sl.symlat.load().sl_autotune_forget()
    recipes = _runs("f64", [32, 48])
    mixed = [sl.from_recipe(r) for r in recipes]
    alone = [sl.from_recipe(r) for r in recipes]
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    b.step(6, 0.005, 4)
    for a in alone:
        a.evolve(6, 0.005, 4)
    tile = mixed[1].tile()
    new = (1.0, 0.5 * recipes[1]["params"][1])
    mixed[1].set_potential("chaotic2", new)
    alone[1].set_potential("chaotic2", new)
    assert mixed[1].tile() == tile
    with pytest.raises(sl.SymlatError) as e:
        mixed[0].set_potential("free", (1.0, 1.0))
    assert e.value.status == 4   # SL_E_STATE
    b.step(9, 0.005, 4)
    for a in alone:
        a.evolve(9, 0.005, 4)
    for j in range(2):
        assert _same(alone[j], mixed[j]), j
    b.close()
