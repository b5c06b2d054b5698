"""CPU model of the Gamma chain sweep kernel's schedule (chain_sweep_kernel in
kpm_chain.hip: KS Chebyshev levels per launch, one stored block row per
level; eq. Gammanm, Sec. 3(b) tiles).

The kernel shares the DOS sweep kernel's row schedule (skewed levels, 4-slot
LDS rings, one barrier per row) but differs in what the model must check
again: one thread per orbital with both spins of a site in each ring cell,
site data and v_{n-1} prefetched with the next row and shifted into the
history at the end of a row (level l reads entry 2 l - 3), ring stores of
threads without a cell redirected to a spare cell, and per-level stores:
the level's block row (mode 0, the L chain), or the velocity of the level
below it from the same neighbour reads (mode 1, the R chain), and the vector
when the level is one of the sweep's last two.

The replay restates the kernel's index arithmetic with symbolic values and
checks, for every configuration: each read of a thread inside a level's
column range (neighbours of both spins against the oracle Hamiltonian's
couplings, the centre, the w term, the site data); LDS bounds against the
allocated rings plus the spare cell; no write by another thread between two
barriers to a cell such a read uses; and exactly-once coverage of every
block row the chain needs (rows 1..nlev in mode 0, 0..nlev-1 in mode 1) and
of the two stored levels, for every orbital and chunk.
"""
import itertools

import pytest

import workload as wl
from oracle import lattice as olat

HONEYCOMB, SPIN, SQUARE = wl.HONEYCOMB, wl.HONEYCOMB_SPIN, wl.SQUARE
NSUB = {HONEYCOMB: 2, SPIN: 2, SQUARE: 1}
NSPIN = {HONEYCOMB: 1, SPIN: 2, SQUARE: 1}
NNB = {HONEYCOMB: 3, SPIN: 3, SQUARE: 4}
_NB = {}


def neighbours(kind, L1, L2):
    """Orbital neighbour sets from the oracle Hamiltonian (Rashba on for the spinful
    lattice, so that both spins of a neighbour couple)."""
    key = (kind, L1, L2)
    if key not in _NB:
        lat = wl.Lattice(kind=kind, L1=L1, L2=L2, t=1.0, rashba=0.3 if kind == SPIN else 0.0)
        H = olat.build(lat).H.tocoo()
        nb = {}
        for i, j, v in zip(H.row, H.col, H.data):
            if i != j and v != 0:
                nb.setdefault(int(i), set()).add(int(j))
        _NB[key] = nb
    return _NB[key]


class Fail(AssertionError):
    pass


def _ult(a, b):
    """(uint32_t)a < (uint32_t)b: a negative a wraps to a large value."""
    return (a & 0xFFFFFFFF) < (b & 0xFFFFFFFF)


def kernel_branches(KS, nlev, ty, j):
    """The kernel's own forms of a row's uniform conditions: level l (2..KS)
    works while j - (3 l - 1 - KS), as a 32-bit unsigned value, is below a
    per-tile count (0 for levels above nlev), level 1 while j <= ty + KS - 1;
    the row a level forms is one of the tile's while j - (2 l - 1) is below ty."""
    lev_cnt = {lev: (ty + 2 * KS - 2 * lev) if lev <= nlev else 0 for lev in range(2, KS + 1)}
    active = {lev: _ult(j - (3 * lev - 1 - KS), lev_cnt[lev]) for lev in range(2, KS + 1)}
    active[1] = j <= ty + KS - 1
    in_tile = {lev: _ult(j - (2 * lev - 1), ty) for lev in range(1, KS + 1)}
    return active, in_tile


def simulate(kind, KS, nlev, mode, block, Ew, E, L1, L2, Ty, g, x0, y0, nb, blk, vec):
    ns, nsp = NSUB[kind], NSPIN[kind]
    Tx = block // (ns * nsp * Ew)
    n_grp = block // Ew
    NH = 2 * KS - 2
    row0 = (Tx + 2) * ns * nsp * Ew
    size = (4 * KS * (Tx + 2) + 1) * ns * nsp * Ew
    lds = ["G"] * size
    writers, readers = {}, {}

    def check(c, msg):
        if not c:
            raise Fail(f"kind {kind} KS {KS} nlev {nlev} mode {mode} block {block} Ew {Ew} E {E} L {L1}x{L2} "
                       f"Ty {Ty} tile ({g},{x0},{y0}): {msg}")

    def write(i, t, v):
        check(0 <= i < size, f"LDS write {i} outside {size}")
        writers.setdefault(i, set()).add(t["tid"])
        lds[i] = v

    def read(i, t, valid):
        check(0 <= i < size, f"LDS read {i} outside {size}")
        if valid:
            readers.setdefault(i, set()).add(t["tid"])
        return lds[i]

    def barrier():
        for i, ws in writers.items():
            rs = readers.get(i, set())
            check(not (rs and (ws - rs or len(ws) > 1 or rs - ws)), f"LDS cell {i}: writers {ws} readers {rs}")
            if len(ws) > 1:
                lds[i] = "X"
        writers.clear()
        readers.clear()

    n_in = min(Tx - 2 * (KS - 1), L1 - x0)
    wcols = n_in + 2 * (KS - 1)
    xe = (x0 - (KS - 1)) % L1
    hl = L1 - 1 if xe == 0 else xe - 1
    hr = (xe + wcols) % L1
    th = []
    for tid in range(block):
        cl, grp = tid % Ew, tid // Ew
        t = dict(tid=tid, cl=cl, grp=grp, sp=(grp // ns) % nsp, s=grp % ns, xl=grp // (ns * nsp))
        t["xlc"] = t["xl"] if grp < n_grp else Tx
        t["n1"] = (xe + t["xl"]) % L1
        t["c"] = g * Ew + cl
        t["ok"] = grp < n_grp and t["c"] < E
        t["act"] = t["ok"] and t["xl"] < wcols
        t["inner"] = t["act"] and KS - 1 <= t["xl"] <= wcols - KS
        t["ll"] = t["ok"] and t["xl"] == 0 and (kind == SQUARE or t["s"] == 0)
        t["lr"] = t["ok"] and t["xl"] == wcols - 1 and (kind == SQUARE or t["s"] == 1)
        t["lh"] = t["ll"] or t["lr"]
        t["hcol"] = hl if t["ll"] else hr
        t["hcell"] = 0 if t["ll"] else wcols + 1
        t["own"], t["halo"], t["w"], t["site"] = [None, None], [None, None], [None, None], [None, None]
        t["hist"] = ["site-init"] * NH
        th.append(t)

    def r0(t, slot, cell, sub, sp):
        return slot * row0 + ((cell * ns + sub) * nsp + sp) * Ew + t["cl"]

    def rl(t, lev, slot, cell, sub, sp):
        return 4 * row0 + ((lev - 1) * 4 + slot) * row0 + ((cell * ns + sub) * nsp + sp) * Ew + t["cl"]

    def spare(t):
        return 4 * KS * row0 + (t["s"] * nsp + t["sp"]) * Ew + t["cl"]

    ty = min(Ty, L2 - y0)
    j0, j_last = 2 - KS, ty + 2 * KS - 2
    wrap = lambda y: y % L2
    nxt = lambda y: 0 if y + 1 == L2 else y + 1

    def fetch(t, k, yv, ysd, inr):
        t["own"][k] = (0, yv, t["n1"], t["s"], t["sp"]) if inr and t["act"] else "0"
        t["halo"][k] = (0, yv, t["hcol"], t["s"], t["sp"]) if inr and t["lh"] else "0"
        in1 = inr and t["act"]
        t["w"][k] = (-1, ysd, t["n1"], t["s"], t["sp"]) if in1 else "0"
        t["site"][k] = ("site", ysd, t["n1"], t["s"]) if in1 else "0"

    def store_row(t, k, slot):
        write(r0(t, slot, t["xl"] + 1, t["s"], t["sp"]) if t["act"] else spare(t), t, t["own"][k])
        write(r0(t, slot, t["hcell"], t["s"], t["sp"]) if t["lh"] else spare(t), t, t["halo"][k])

    def cells(t, x, s0, sp1, sm1):
        if kind == SQUARE:
            return [(s0, x + 1, 0), (s0, x - 1, 0), (sp1, x, 0), (sm1, x, 0)]
        if t["s"] == 0:
            return [(s0, x, 1), (sm1, x + 1, 1), (sm1, x, 1)]
        return [(s0, x, 0), (sp1, x - 1, 0), (sp1, x, 0)]

    def orb(row, col, sub, sp):
        return ((row * L1 + col) * ns + sub) * nsp + sp

    def check_step(t, lev, y, vn, vo, wo, site):
        yw = wrap(y)
        me = (yw, t["n1"], t["s"], t["sp"])
        check(vo == (lev - 1,) + me, f"level {lev} row {y}: centre {vo}")
        check(wo == (lev - 2,) + me, f"level {lev} row {y}: w {wo}")
        check(site == ("site", yw, t["n1"], t["s"]), f"level {lev} row {y}: site {site}")
        got = []
        for v in vn:
            check(isinstance(v, tuple) and v[0] == lev - 1, f"level {lev} row {y}: neighbour {v}")
            got.append(orb(*v[1:]))
        check(set(got) == nb[orb(*me)], f"level {lev} row {y}: neighbours {sorted(got)} vs {sorted(nb[orb(*me)])}")
        if L1 >= 3 and L2 >= 3:
            check(len(set(got)) == NNB[kind] * nsp, f"repeated neighbour {got}")

    def emit(t, lev, yw, own, o, gv):
        if not own:
            return
        key = (t["n1"], t["s"], t["sp"], t["c"])
        if mode == 0:
            check(o == (lev, yw, t["n1"], t["s"], t["sp"]), f"block value {o}")
            k = (lev, yw) + key
        else:
            check(gv == ("vel", lev - 1, yw, t["n1"], t["s"], t["sp"]), f"block velocity {gv}")
            k = (lev - 1, yw) + key
        check(k not in blk, f"second block store {k}")
        blk[k] = 1
        if lev in (nlev, nlev - 1):
            kv = ("b" if lev == nlev else "a", yw) + key
            check(kv not in vec, f"second vector store {kv}")
            check(o == (lev, yw, t["n1"], t["s"], t["sp"]), f"vector value {o}")
            vec[kv] = 1

    for t in th:
        fetch(t, 0, wrap(y0 - KS), wrap(y0 - KS), True)
        store_row(t, 0, 0)
        fetch(t, 1, wrap(y0 - KS + 1), wrap(y0 - KS + 1), True)
        store_row(t, 1, 1)
        fetch(t, 0, wrap(y0 + j0), wrap(y0 + j0 - 1), True)
    regs = {"yf": wrap(y0 + j0 + 1), "ys": wrap(y0 + j0)}
    yl = {l: wrap(y0 + j0 - (2 * l - 1)) for l in range(1, KS + 1)}

    def row(p, j):
        for t in th:
            store_row(t, p & 1, (p + 2) & 3)
            t["w1"], t["s1"] = t["w"][p & 1], t["site"][p & 1]
            fetch(t, (p + 1) & 1, regs["yf"], regs["ys"], j + 1 <= ty + KS - 1)
        # The kernel's unsigned forms of the conditions below agree with them.
        k_active, k_in_tile = kernel_branches(KS, nlev, ty, j)
        for lev in range(1, KS + 1):
            lo = 3 * lev - 1 - KS if lev >= 2 else j0
            check(k_active[lev] == (lev <= nlev and lo <= j <= ty + KS + lev - 2), f"level {lev} activity at j={j}")
            check(k_in_tile[lev] == (y0 <= y0 + j - (2 * lev - 1) < y0 + ty), f"level {lev} row in tile at j={j}")
        barrier()
        for t in th:
            x = t["xlc"] + 1
            for lev in range(KS, 1, -1):
                y = y0 + j - (2 * lev - 1)
                if not (lev <= nlev and 3 * lev - 1 - KS <= j <= ty + KS + lev - 2):
                    continue
                valid = t["ok"] and lev - 1 <= t["xl"] <= wcols - lev
                sp1, s0, sm1 = (p + 3) & 3, (p + 2) & 3, (p + 1) & 3
                vn = [read(rl(t, lev - 1, sl, cell, sub, sp), t, valid)
                      for sl, cell, sub in cells(t, x, s0, sp1, sm1) for sp in range(nsp)]
                vo = read(rl(t, lev - 1, s0, x, t["s"], t["sp"]), t, valid)
                wo = read(r0(t, (p + 3) & 3, x, t["s"], t["sp"]) if lev == 2 else
                          rl(t, lev - 2, p, x, t["s"], t["sp"]), t, valid)
                if valid:
                    check_step(t, lev, y, vn, vo, wo, t["hist"][2 * lev - 3])
                    o = (lev, wrap(y), t["n1"], t["s"], t["sp"])
                    gv = ("vel", lev - 1, wrap(y), t["n1"], t["s"], t["sp"])
                else:
                    o = gv = "G"
                if lev < KS:
                    write(rl(t, lev, p, x, t["s"], t["sp"]), t, o)
                check(yl[lev] == wrap(y), f"row register of level {lev}")
                emit(t, lev, yl[lev], t["inner"] and y0 <= y < y0 + ty, o, gv)
            if j <= ty + KS - 1:
                y = y0 + j - 1
                valid = t["ok"] and 0 <= t["xl"] <= wcols - 1
                sp1, s0, sm1 = (p + 2) & 3, (p + 1) & 3, p
                vn = [read(r0(t, sl, cell, sub, sp), t, valid) for sl, cell, sub in cells(t, x, s0, sp1, sm1)
                      for sp in range(nsp)]
                vo = read(r0(t, s0, x, t["s"], t["sp"]), t, valid)
                if valid:
                    check_step(t, 1, y, vn, vo, t["w1"], t["s1"])
                    o = (1, wrap(y), t["n1"], t["s"], t["sp"])
                    gv = ("vel", 0, wrap(y), t["n1"], t["s"], t["sp"])
                else:
                    o = gv = "G"
                write(rl(t, 1, p, x, t["s"], t["sp"]), t, o)
                check(yl[1] == wrap(y), "row register of level 1")
                emit(t, 1, yl[1], t["inner"] and y0 <= y < y0 + ty, o, gv)
            t["hist"] = [t["s1"]] + t["hist"][:-1]
        regs["yf"], regs["ys"] = nxt(regs["yf"]), nxt(regs["ys"])
        for l in yl:
            yl[l] = nxt(yl[l])

    j = j0
    while j <= j_last:
        for p in range(4):
            row(p, j + p)
        j += 4
    barrier()


def run(kind, KS, nlev, mode, block, Ew, E, L1, L2, Ty):
    ns, nsp = NSUB[kind], NSPIN[kind]
    Tx = block // (ns * nsp * Ew)
    assert Tx >= 2 * KS - 1
    xstep = Tx - 2 * (KS - 1)
    nb = neighbours(kind, L1, L2)
    blk, vec = {}, {}
    for g in range(-(-E // Ew)):
        for y0 in range(0, L2, Ty):
            for x0 in range(0, L1, xstep):
                simulate(kind, KS, nlev, mode, block, Ew, E, L1, L2, Ty, g, x0, y0, nb, blk, vec)
    rows = range(1, nlev + 1) if mode == 0 else range(0, nlev)
    keys = [(r, y, x, s, sp, c) for r in rows for y in range(L2) for x in range(L1) for s in range(ns)
            for sp in range(nsp) for c in range(E)]
    assert len(blk) == len(keys) and all(k in blk for k in keys), (kind, KS, nlev, mode)
    n_vec = (2 if nlev >= 2 else 1) * L2 * L1 * ns * nsp * E
    assert len(vec) == n_vec


# (block, Ew, E): exact fits, surplus threads and a partial column (block not a multiple of
# NSUB * NSPIN * Ew), idle lanes in the last r-group (E not a multiple of Ew).
SHAPES = [(64, 1, 1), (64, 2, 3), (192, 5, 5), (128, 2, 2)]


def configs():
    out = []
    for kind, KS in itertools.product((SPIN, HONEYCOMB, SQUARE), (2, 3, 4)):
        for block, Ew, E in SHAPES:
            Tx = block // (NSUB[kind] * NSPIN[kind] * Ew)
            if Tx < 2 * KS - 1:
                continue
            xstep = Tx - 2 * (KS - 1)
            lats = [(2, 3, 2), (min(xstep, 6), 5, 3), (xstep + 2, 4, 8)]
            for nlev in range(1, KS + 1):
                for mode in (0, 1):
                    for L1, L2, Ty in (lats if nlev == KS else lats[1:2]):
                        if L1 >= 2:
                            out.append((kind, KS, nlev, mode, block, Ew, E, L1, L2, Ty))
    return out


CONFIGS = configs()


def test_chain_schedule_configurations():
    assert len(CONFIGS) >= 150
    assert {c[0] for c in CONFIGS} == {SPIN, HONEYCOMB, SQUARE}
    assert any(c[2] < c[1] for c in CONFIGS) and {c[3] for c in CONFIGS} == {0, 1}


@pytest.mark.parametrize("kind", [SPIN, HONEYCOMB, SQUARE], ids=["spin", "honeycomb", "square"])
def test_chain_schedule(kind):
    n = 0
    for cfg in CONFIGS:
        if cfg[0] == kind:
            run(*cfg)
            n += 1
    assert n > 0


def test_chain_model_detects_planted_mistakes():
    """A wrong site-history entry, ring slot for w, or store row in the replay fails it."""
    global simulate
    import inspect
    src = inspect.getsource(simulate)
    mutants = [
        ('t["hist"][2 * lev - 3]', 't["hist"][2 * lev - 2]'),
        ("rl(t, lev - 2, p, x, t[\"s\"], t[\"sp\"])", "rl(t, lev - 2, (p + 2) & 3, x, t[\"s\"], t[\"sp\"])"),
        ("k = (lev - 1, yw) + key", "k = (lev, yw) + key"),
        ('(sm1, x + 1, 1), (sm1, x, 1)]', '(sm1, x - 1, 1), (sm1, x, 1)]'),
    ]
    original = simulate
    try:
        for a, b in mutants:
            assert a in src, a
            ns = {}
            exec(compile(src.replace(a, b), "<mutant>", "exec"), globals(), ns)
            simulate = ns["simulate"]
            with pytest.raises(AssertionError):
                run(SPIN, 3, 3, 1, 64, 1, 1, 6, 5, 3)
            simulate = original
    finally:
        simulate = original


def test_chain_model_detects_planted_branch_mistakes():
    """A level count one too large or a tile-row check off by one in the
    kernel's unsigned forms fails the model."""
    global kernel_branches
    import inspect
    src = inspect.getsource(kernel_branches)
    mutants = [
        ("(ty + 2 * KS - 2 * lev) if", "(ty + 2 * KS - 2 * lev + 1) if"),
        ("_ult(j - (2 * lev - 1), ty)", "_ult(j - (2 * lev - 2), ty)"),
    ]
    original = kernel_branches
    try:
        for a, b in mutants:
            assert a in src, a
            ns = {}
            exec(compile(src.replace(a, b), "<mutant>", "exec"), globals(), ns)
            kernel_branches = ns["kernel_branches"]
            with pytest.raises(AssertionError):
                run(SPIN, 3, 3, 1, 64, 1, 1, 6, 5, 3)
            kernel_branches = original
    finally:
        kernel_branches = original
