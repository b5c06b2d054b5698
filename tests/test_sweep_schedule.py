"""CPU model of the temporally blocked sweep kernel's schedule (sweep_kernel in
kpm_sweep.hip: KS Chebyshev steps per launch over one tile, Sec. 3(b) tiles).

The model replays tiles of the kernel thread by thread with the kernel's own
index arithmetic restated: the thread -> (chunk, sublattice, thread column)
map, the tile's columns and halos, the row registers and their wrap, the
prologue, the 4-row unrolled loop with its ring slots, the level ranges, the
register history of site data, the two stores of a row and the
element-wise selects of the stored levels.  LDS and registers hold symbolic
tags (level, row, column, sublattice) instead of numbers.  For every
configuration it checks that

* every value a thread inside a level's column range reads is the one that
  step needs: the previous level at the site and at the neighbours that the
  oracle's Hamiltonian couples to it (so the stencil is the paper's lattice,
  honeycomb bonds of Sec. 3(d) or the square lattice), the level before that
  at the site (the w term), and the site data of that row;
* every LDS index is inside the rings the plan allocates;
* no LDS cell that such a read uses is written by another thread between the
  same two barriers;
* every site of the lattice (and every chunk of vectors) receives the two
  stored levels exactly once over the tile list, with the right level, and
  every level's dot products count each site exactly once.

Shapes cover KS = 2..5, short last sweeps (nlev < KS), honeycomb and square
lattices, workgroups whose size is not a multiple of the columns (surplus
threads and a partial column), chunk counts that leave idle lanes in the last
r-group, lattices narrower than a tile's halo span, and ragged row bands.
"""
import itertools
from collections import Counter

import numpy as np
import pytest

import workload as wl
from oracle import lattice as olat

HONEYCOMB, SQUARE = wl.HONEYCOMB, wl.SQUARE
NNB = {HONEYCOMB: 3, SQUARE: 4}
NSUBS = {HONEYCOMB: 2, SQUARE: 1}

_NB_CACHE = {}


def oracle_neighbours(kind, L1, L2):
    """Neighbour sets of every site from the oracle's sparse Hamiltonian (no disorder)."""
    key = (kind, L1, L2)
    if key not in _NB_CACHE:
        m = olat.build(wl.Lattice(kind=kind, L1=L1, L2=L2, t=1.0))
        H = m.H.tocoo()
        nb = {}
        for i, j, v in zip(H.row, H.col, H.data):
            if i != j and v != 0:
                nb.setdefault(int(i), set()).add(int(j))
        _NB_CACHE[key] = nb
    return _NB_CACHE[key]


class ScheduleError(AssertionError):
    pass


class Thread:
    __slots__ = ("tid", "cl", "grp", "s", "xl", "xlc", "n1", "c", "lane_ok", "act", "inner", "load_left",
                 "load_right", "load_halo", "halo_col", "halo_cell", "sets", "ons_h", "o_a", "o_b")


def tile_list(L1, L2, Tx, Ty, KS, n_rg):
    """The plan's tile list for one lattice: (r-group, x0, y0), x0 stepping by the interior width."""
    xstep = Tx - 2 * (KS - 1)
    return [(g, x0, y0) for g in range(n_rg) for y0 in range(0, L2, Ty) for x0 in range(0, L1, xstep)]


def _ult(a, b):
    """(uint32_t)a < (uint32_t)b: a negative a wraps to a large value."""
    return (a & 0xFFFFFFFF) < (b & 0xFFFFFFFF)


def kernel_branches(KS, nlev, ty, j):
    """The kernel's own forms of a row's uniform conditions: per-tile counts
    and 32-bit unsigned comparisons, and in a full sweep (nlev == KS, its own
    compile-time branch) the fixed stored levels.  Returns the activity of
    levels 1..KS, whether the row each level forms lies in the tile, and the
    row parts of the two store checks."""
    full = nlev == KS
    nl = KS if full else nlev
    lev_cnt = {lev: (ty + 2 * KS - 2 * lev) if lev <= nlev else 0 for lev in range(2, KS + 1)}
    a_cnt = ty if nlev >= 2 else 0
    active = {lev: _ult(j - (3 * lev - 1 - KS), lev_cnt[lev]) for lev in range(2, KS + 1)}
    active[1] = j <= ty + KS - 1
    in_tile = {lev: _ult(j - (2 * lev - 1), ty) for lev in range(1, KS + 1)}
    own_b = _ult(j - (2 * nl - 1), ty)
    own_a = _ult(j - (2 * nl - 3), ty if full else a_cnt)
    return active, in_tile, own_b, own_a


def simulate_tile(kind, KS, nlev, block, Ew, E, L1, L2, Ty, g, x0, y0, nb, stores, dots):
    NSUB = NSUBS[kind]
    Tx = block // (NSUB * Ew)
    n_grp = block // Ew
    NH = 2 * KS - 1
    row0 = (Tx + 2) * NSUB * Ew
    lds_size = (4 * KS * (Tx + 2) + 1) * NSUB * Ew   # the rings the plan allocates (16-byte packs)
    lds = ["G"] * lds_size
    iv_writers, iv_readers = {}, {}

    def check(cond, msg):
        if not cond:
            raise ScheduleError(f"kind {kind} KS {KS} nlev {nlev} block {block} Ew {Ew} E {E} L {L1}x{L2} "
                                f"Ty {Ty} tile (g {g}, x0 {x0}, y0 {y0}): {msg}")

    def r0(slot, cell, sub, cl):
        return slot * row0 + (cell * NSUB + sub) * Ew + cl

    def rl(lev, slot, cell, sub, cl):
        return 4 * row0 + ((lev - 1) * 4 + slot) * row0 + (cell * NSUB + sub) * Ew + cl

    def write(idx, t, tag):
        check(0 <= idx < lds_size, f"LDS write {idx} outside [0, {lds_size})")
        iv_writers.setdefault(idx, set()).add(t.tid)
        lds[idx] = tag

    def read(idx, t, valid):
        check(0 <= idx < lds_size, f"LDS read {idx} outside [0, {lds_size})")
        if valid:
            iv_readers.setdefault(idx, set()).add(t.tid)
        return lds[idx]

    def barrier():
        for idx, ws in iv_writers.items():
            rs = iv_readers.get(idx, set())
            check(not (rs and (ws - rs or len(ws) > 1 or rs - ws)),
                  f"LDS cell {idx}: written by {sorted(ws)} and read by {sorted(rs)} between two barriers")
            if len(ws) > 1:
                lds[idx] = "X"   # several writers: the value is undetermined
        iv_writers.clear()
        iv_readers.clear()

    n_in = min(Tx - 2 * (KS - 1), L1 - x0)
    wcols = n_in + 2 * (KS - 1)
    xe = (x0 - (KS - 1)) % L1
    hl = L1 - 1 if xe == 0 else xe - 1
    hr = (xe + wcols) % L1
    threads = []
    for tid in range(block):
        t = Thread()
        t.tid = tid
        t.cl = tid % Ew
        t.grp = tid // Ew
        t.s = t.grp % NSUB
        t.xl = t.grp // NSUB
        t.xlc = t.xl if t.grp < n_grp else Tx
        t.n1 = (xe + t.xl) % L1
        t.c = g * Ew + t.cl
        t.lane_ok = t.grp < n_grp and t.c < E
        t.act = t.lane_ok and t.xl < wcols
        t.inner = t.act and KS - 1 <= t.xl <= wcols - KS
        t.load_left = t.lane_ok and t.xl == 0 and (kind == SQUARE or t.s == 0)
        t.load_right = t.lane_ok and t.xl == wcols - 1 and (kind == SQUARE or t.s == 1)
        t.load_halo = t.load_left or t.load_right
        t.halo_col = hl if t.load_left else hr
        t.halo_cell = 0 if t.load_left else wcols + 1
        t.sets = [None, None]
        t.ons_h = ["site-init"] * NH
        t.o_a = t.o_b = "stale"
        threads.append(t)

    ty = min(Ty, L2 - y0)
    j0 = 2 - KS
    j_last = ty + 2 * KS - 2

    def wrap(y):
        return y % L2

    def next_row(y):
        return 0 if y + 1 == L2 else y + 1

    def fetch(t, yv, ys, in_range):
        own = (0, yv, t.n1, t.s) if in_range and t.act else "0"
        halo = (0, yv, t.halo_col, t.s) if in_range and t.load_halo else "0"
        w = (-1, ys, t.n1, t.s) if in_range and t.act else "0"
        site = ("site", ys, t.n1, t.s) if in_range and t.act else "0"
        return [own, halo, w, site]

    def fetch_v(t, yv):
        return [(0, yv, t.n1, t.s) if t.act else "0", (0, yv, t.halo_col, t.s) if t.load_halo else "0", None, None]

    def store_row(t, S, slot):
        if t.act:
            write(r0(slot, t.xl + 1, t.s, t.cl), t, S[0])
        if t.load_halo:
            write(r0(slot, t.halo_cell, t.s, t.cl), t, S[1])

    def neighbour_cells(t, x, s0, sp1, sm1):
        """(slot, cell, sub) of the NNB neighbours, as the kernel reads them."""
        if kind == SQUARE:
            return [(s0, x + 1, 0), (s0, x - 1, 0), (sp1, x, 0), (sm1, x, 0)]
        if t.s == 0:
            return [(s0, x, 1), (sm1, x + 1, 1), (sm1, x, 1)]
        return [(s0, x, 0), (sp1, x - 1, 0), (sp1, x, 0)]

    def check_step(t, lev, y, vn_tags, vo, wo, site):
        """Inputs of level lev at unwrapped row y for a thread inside the level's columns."""
        yw = wrap(y)
        me = (yw * L1 + t.n1) * NSUB + t.s
        check(vo == (lev - 1, yw, t.n1, t.s), f"level {lev} row {y} col {t.n1}: centre {vo}")
        check(wo == (lev - 2, yw, t.n1, t.s), f"level {lev} row {y} col {t.n1}: w term {wo}")
        check(site == ("site", yw, t.n1, t.s), f"level {lev} row {y} col {t.n1}: site data {site}")
        got = []
        for tag in vn_tags:
            check(isinstance(tag, tuple) and tag[0] == lev - 1,
                  f"level {lev} row {y} col {t.n1} sub {t.s}: neighbour {tag}")
            got.append((tag[1] * L1 + tag[2]) * NSUB + tag[3])
        check(set(got) == nb[me], f"level {lev} row {y} col {t.n1} sub {t.s}: neighbours {got} vs {nb[me]}")
        if L1 >= 3 and L2 >= 3:
            check(len(set(got)) == NNB[kind], f"level {lev}: repeated neighbour {got}")

    def row(p, j):
        yf, ys, yb, ya = regs
        # store_row of the arrived set, shift of the site history, fetch of the next row.
        for t in threads:
            cur = t.sets[p % 2]
            store_row(t, cur, (p + 2) & 3)
            t.ons_h = [cur[3]] + t.ons_h[:-1]
            t.sets[(p + 1) % 2] = fetch(t, yf, ys, j + 1 <= ty + KS - 1)
        check(yf == wrap(y0 + j + 1) and ys == wrap(y0 + j), f"row registers at j={j}")
        # The kernel's unsigned forms of the conditions below agree with them.
        k_active, k_in_tile, k_own_b, k_own_a = kernel_branches(KS, nlev, ty, j)
        for lev in range(1, KS + 1):
            lo = 3 * lev - 1 - KS if lev >= 2 else j0
            hi = ty + KS + lev - 2
            check(k_active[lev] == (lev <= nlev and lo <= j <= hi), f"level {lev} activity at j={j}")
            yl = y0 + j - (2 * lev - 1)
            check(k_in_tile[lev] == (y0 <= yl < y0 + ty), f"level {lev} row in tile at j={j}")
        yb_u = y0 + j - (2 * nlev - 1)
        check(k_own_b == (y0 <= yb_u < y0 + ty), f"store b at j={j}")
        check(k_own_a == (nlev >= 2 and y0 <= yb_u + 2 < y0 + ty), f"store a at j={j}")
        barrier()
        for t in threads:
            x = t.xlc + 1
            cur = t.sets[p % 2]
            for lev in range(KS, 1, -1):
                y = y0 + j - (2 * lev - 1)
                if not (lev <= nlev and 3 * lev - 1 - KS <= j <= ty + KS + lev - 2):
                    continue
                valid = t.lane_ok and lev - 1 <= t.xl <= wcols - lev
                sp1, s0, sm1 = (p + 3) & 3, (p + 2) & 3, (p + 1) & 3
                vn = [read(rl(lev - 1, sl, cell, sub, t.cl), t, valid)
                      for sl, cell, sub in neighbour_cells(t, x, s0, sp1, sm1)]
                vo = read(rl(lev - 1, s0, x, t.s, t.cl), t, valid)
                if lev == 2:
                    wo = read(r0((p + 3) & 3, x, t.s, t.cl), t, valid)
                else:
                    wo = read(rl(lev - 2, p, x, t.s, t.cl), t, valid)
                if valid:
                    check_step(t, lev, y, vn, vo, wo, t.ons_h[2 * lev - 2])
                    o = (lev, wrap(y), t.n1, t.s)
                else:
                    o = "G"
                if t.inner and y0 <= y < y0 + ty:
                    dots[(lev, wrap(y), t.n1, t.s, t.c)] += 1
                if lev < KS:
                    write(rl(lev, p, x, t.s, t.cl), t, o)
                if lev == KS:
                    t.o_b = o
                if lev == KS - 1:
                    t.o_a = o
                if nlev < KS:
                    if lev == nlev:
                        t.o_b = o
                    if lev == nlev - 1:
                        t.o_a = o
            # Level 1.
            y = y0 + j - 1
            if j <= ty + KS - 1:
                valid = t.lane_ok and 0 <= t.xl <= wcols - 1
                sp1, s0, sm1 = (p + 2) & 3, (p + 1) & 3, p
                vn = [read(r0(sl, cell, sub, t.cl), t, valid) for sl, cell, sub in neighbour_cells(t, x, s0, sp1, sm1)]
                vo = read(r0(s0, x, t.s, t.cl), t, valid)
                if valid:
                    check_step(t, 1, y, vn, vo, cur[2], t.ons_h[0])
                    o = (1, wrap(y), t.n1, t.s)
                else:
                    o = "G"
                if t.inner and y0 <= y < y0 + ty:
                    dots[(1, wrap(y), t.n1, t.s, t.c)] += 1
                write(rl(1, p, x, t.s, t.cl), t, o)
                if KS == 2:
                    t.o_a = o
                if nlev <= 2:
                    if nlev == 1:
                        t.o_b = o
                    else:
                        t.o_a = o
            # The row's two stores.
            yb_u = y0 + j - (2 * nlev - 1)
            own_b = t.inner and y0 <= yb_u < y0 + ty
            own_a = t.inner and nlev >= 2 and y0 <= yb_u + 2 < y0 + ty
            if own_b:
                check(yb == wrap(yb_u), f"store row register {yb} vs {wrap(yb_u)}")
                check(t.o_b == (nlev, wrap(yb_u), t.n1, t.s), f"stored level {t.o_b} at row {yb_u}")
                key = ("b", yb, t.n1, t.s, t.c)
                check(key not in stores, f"second store of {key}")
                stores[key] = t.o_b
            if own_a:
                check(ya == wrap(yb_u + 2), f"store row register {ya} vs {wrap(yb_u + 2)}")
                check(t.o_a == (nlev - 1, wrap(yb_u + 2), t.n1, t.s), f"stored level {t.o_a} at row {yb_u + 2}")
                key = ("a", ya, t.n1, t.s, t.c)
                check(key not in stores, f"second store of {key}")
                stores[key] = t.o_a
        regs[:] = [next_row(yf), next_row(ys), next_row(yb), next_row(ya)]

    # Prologue: v_n rows y0 - KS and y0 - KS + 1 into slots 0 and 1, then the first row's loads.
    for t in threads:
        store_row(t, fetch_v(t, wrap(y0 - KS)), 0)
        store_row(t, fetch_v(t, wrap(y0 - KS + 1)), 1)
        t.sets[0] = fetch(t, wrap(y0 + j0), wrap(y0 + j0 - 1), True)
    regs = [wrap(y0 + j0 + 1), wrap(y0 + j0), wrap(y0 + j0 - (2 * nlev - 1)), wrap(y0 + j0 - (2 * nlev - 3))]
    j = j0
    while j <= j_last:
        for p in range(4):
            row(p, j + p)
        j += 4
    barrier()


def run_config(kind, KS, nlev, block, Ew, E, L1, L2, Ty):
    NSUB = NSUBS[kind]
    Tx = block // (NSUB * Ew)
    assert Tx >= 2 * KS - 1, "the plan needs at least 2 KS - 1 thread columns"
    n_rg = -(-E // Ew)
    nb = oracle_neighbours(kind, L1, L2)
    stores, dots = {}, Counter()
    for g, x0, y0 in tile_list(L1, L2, Tx, Ty, KS, n_rg):
        simulate_tile(kind, KS, nlev, block, Ew, E, L1, L2, Ty, g, x0, y0, nb, stores, dots)
    sites = [(y, x, s) for y in range(L2) for x in range(L1) for s in range(NSUB)]
    for buf, lev in (("b", nlev), ("a", nlev - 1)):
        if lev < 1:
            continue
        for (y, x, s) in sites:
            for c in range(E):
                assert stores.get((buf, y, x, s, c)) == (lev, y, x, s), (kind, KS, nlev, buf, y, x, s, c)
    n_expected = sum(1 for lev in range(1, nlev + 1) for _ in sites for _ in range(E))
    assert sum(1 for k in stores) == len(sites) * E * (2 if nlev >= 2 else 1)
    assert len(dots) == n_expected and all(v == 1 for v in dots.values()), (kind, KS, nlev)
    for lev, y, x, s, c in dots:
        assert 1 <= lev <= nlev and c < E


# (block, Ew, E) shapes: exact fits, a partial thread column and surplus threads
# (block not a multiple of NSUB * Ew), idle lanes in the last r-group (E not a
# multiple of Ew).
SHAPES = [(64, 1, 1), (64, 2, 3), (64, 3, 5), (64, 4, 6), (64, 5, 5), (96, 2, 2)]


def _configs():
    out = []
    for kind, KS in itertools.product((HONEYCOMB, SQUARE), (2, 3, 4, 5)):
        for block, Ew, E in SHAPES:
            Tx = block // (NSUBS[kind] * Ew)
            if Tx < 2 * KS - 1:
                continue
            xstep = Tx - 2 * (KS - 1)
            # Lattices: narrower than the halo span, one tile wide, ragged; row bands ragged.
            lats = [(2, 3, 2), (min(xstep, 7), 5, 3), (xstep + 3, 4, 8), (2 * xstep - 1, 7, 4)]
            for nlev in range(1, KS + 1):
                for L1, L2, Ty in (lats if nlev == KS else lats[1::2]):
                    if L1 < 2:
                        continue
                    out.append((kind, KS, nlev, block, Ew, E, L1, L2, Ty))
    return out


CONFIGS = _configs()


def test_sweep_schedule_model_covers_configurations():
    assert len(CONFIGS) >= 250
    kinds = {c[0] for c in CONFIGS}
    ks = {c[1] for c in CONFIGS}
    assert kinds == {HONEYCOMB, SQUARE} and ks == {2, 3, 4, 5}
    assert any(c[2] < c[1] for c in CONFIGS)   # short last sweeps


@pytest.mark.parametrize("kind,KS", [(k, s) for k in (HONEYCOMB, SQUARE) for s in (2, 3, 4, 5)])
def test_sweep_schedule(kind, KS):
    n = 0
    for cfg in CONFIGS:
        if cfg[0] == kind and cfg[1] == KS:
            run_config(*cfg)
            n += 1
    assert n > 0


def test_benchmarked_tile_shape():
    """The headline shape: 512 threads, 8 chunks per site, KS = 4 (Tx = 32 on the
    honeycomb lattice), 24 interior columns, one tile wide and a ragged band."""
    run_config(HONEYCOMB, 4, 4, 512, 8, 8, 26, 5, 4)
    run_config(HONEYCOMB, 4, 2, 512, 8, 16, 25, 3, 2)


def test_model_detects_planted_mistakes():
    """The model is not vacuous: a wrong ring slot, level range, halo cell,
    neighbour offset or interior range in the replayed schedule fails it."""
    global simulate_tile
    import inspect
    src = inspect.getsource(simulate_tile)
    mutants = [
        ("sp1, s0, sm1 = (p + 3) & 3, (p + 2) & 3, (p + 1) & 3", "sp1, s0, sm1 = (p + 2) & 3, (p + 3) & 3, (p + 1) & 3"),
        ("3 * lev - 1 - KS <= j", "3 * lev - KS <= j"),
        ("t.halo_cell = 0 if t.load_left else wcols + 1", "t.halo_cell = 0 if t.load_left else wcols"),
        ("[(s0, x, 1), (sm1, x + 1, 1), (sm1, x, 1)]", "[(s0, x, 1), (sm1, x - 1, 1), (sm1, x, 1)]"),
        ("wo = read(rl(lev - 2, p, x, t.s, t.cl), t, valid)", "wo = read(rl(lev - 2, (p + 1) & 3, x, t.s, t.cl), t, valid)"),
        ("t.inner = t.act and KS - 1 <= t.xl <= wcols - KS", "t.inner = t.act and KS - 2 <= t.xl <= wcols - KS"),
    ]
    original = simulate_tile
    try:
        for a, b in mutants:
            assert a in src, a
            ns = {}
            exec(compile(src.replace(a, b), "<mutant>", "exec"), globals(), ns)
            simulate_tile = ns["simulate_tile"]
            with pytest.raises(AssertionError):
                run_config(HONEYCOMB, 4, 4, 64, 1, 1, 7, 5, 3)
                run_config(HONEYCOMB, 3, 2, 64, 2, 3, 9, 4, 8)
            simulate_tile = original
    finally:
        simulate_tile = original


def test_model_detects_planted_branch_mistakes():
    """The kernel's unsigned forms of its row conditions are checked against
    the level ranges: a level count one too large (a level running one
    iteration past its range) or a store check that ignores a one-level
    sweep fails the model."""
    global kernel_branches
    import inspect
    src = inspect.getsource(kernel_branches)
    mutants = [
        ("(ty + 2 * KS - 2 * lev) if", "(ty + 2 * KS - 2 * lev + 1) if"),
        ("_ult(j - (2 * nl - 3), ty if full else a_cnt)", "_ult(j - (2 * nl - 3), ty)"),
    ]
    original = kernel_branches
    try:
        for a, b in mutants:
            assert a in src, a
            ns = {}
            exec(compile(src.replace(a, b), "<mutant>", "exec"), globals(), ns)
            kernel_branches = ns["kernel_branches"]
            with pytest.raises(AssertionError):
                run_config(HONEYCOMB, 4, 4, 64, 1, 1, 7, 5, 3)
                run_config(HONEYCOMB, 3, 1, 64, 2, 3, 9, 4, 8)
            kernel_branches = original
    finally:
        kernel_branches = original
