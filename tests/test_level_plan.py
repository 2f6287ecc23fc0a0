"""The level form's host plan (no GPU): the ghost exchange table that the
library builds for boxes tiling one periodic domain (Sec. 2.6: boxes of a
level couple only through their ghost zones).  Every block is decoded here
and applied to an array of level-cell ids: each ghost position of every box
must be written exactly once, from an interior position of a box, with the id
of the level cell that is congruent to it modulo the domain.  This is also
the bounds check of the exchange kernel's indexing.  Levels that do not tile
their domain are refused."""
import numpy as np
import pytest

from paper_2609_10816_amd import ctmhd

PH_F, PH_E, PH_U, PH_O, PH_X, PH_WRAP, PH_DT, PH_COPY, PH_P, PH_XCHG, PH_FIRST = range(11)
XG_HALF, XG_NEXT, XG_CUR, XG_FLAGS, XG_IF_FIXUP = 0, 1, 2, 4, 8


def _level(domain, cuts, shift, ng):
    """Boxes (packed back to back with gaps), their origins and shapes."""
    boxes, origin, off = [], [], 0
    for k in range(len(cuts[2]) - 1):
        for j in range(len(cuts[1]) - 1):
            for i in range(len(cuts[0]) - 1):
                lo = [cuts[0][i], cuts[1][j], cuts[2][k]]
                n = [cuts[0][i + 1] - lo[0], cuts[1][j + 1] - lo[1], cuts[2][k + 1] - lo[2]]
                boxes.append(ctmhd.make_box(n, ng, (0.1, 0.1, 0.1), off))
                origin.append([(lo[d] + shift[d]) % domain[d] for d in range(3)])
                off += int(np.prod([v + 2 * ng for v in n])) + 7 * len(boxes)
    return boxes, np.asarray(origin, np.int32), off


def _apply(d, boxes, origin, total):
    """Level-cell ids in every interior position, then every exchange block."""
    ids = np.full(total, -1, np.int64)
    owner = np.full(total, -1, np.int64)  # box whose interior holds a position
    for b, bx in enumerate(boxes):
        g, n = bx.ng, list(bx.n)
        N = [v + 2 * g for v in n]
        k, j, i = np.meshgrid(np.arange(g, g + n[2]), np.arange(g, g + n[1]), np.arange(g, g + n[0]),
                              indexing="ij")
        pos = bx.offset + i + N[0] * (j + N[1] * k)
        lev = [(origin[b][d] + (c - g)) % DOMAIN[d] for d, c in enumerate((i, j, k))]
        ids[pos] = lev[0] + DOMAIN[0] * (lev[1] + DOMAIN[1] * lev[2])
        owner[pos] = b
    writes = np.zeros(total, np.int64)
    out = ids.copy()
    for b, bx in enumerate(boxes):
        vol = 0
        for q in range(d["xbox"][b], d["xbox"][b + 1]):
            e = d["xblk"][q]
            assert e["vol_lo"] == vol
            vol += int(e["vol"])
            ez = int(e["vol"]) // (int(e["ex"]) * int(e["ey"]))
            assert ez * int(e["ex"]) * int(e["ey"]) == int(e["vol"])
            z, y, x = np.meshgrid(np.arange(ez), np.arange(e["ey"]), np.arange(e["ex"]), indexing="ij")
            dst = int(e["dst"]) + x + int(e["dsy"]) * y + int(e["dsz"]) * z
            src = int(e["src"]) + x + int(e["ssy"]) * y + int(e["ssz"]) * z
            assert dst.min() >= bx.offset and dst.max() < bx.offset + ctmhd.lib().ctmhd_box_elems(bx)
            assert (owner[src] >= 0).all(), "an exchange source is not an interior position"
            assert (owner[dst] == -1).all(), "an exchange writes an interior position"
            out[dst.ravel()] = ids[src.ravel()]
            np.add.at(writes, dst.ravel(), 1)
        assert vol == ctmhd.lib().ctmhd_box_elems(bx) - int(np.prod(bx.n))
    return out, writes


def _expected(boxes, origin, total):
    exp = np.full(total, -1, np.int64)
    for b, bx in enumerate(boxes):
        g, n = bx.ng, list(bx.n)
        N = [v + 2 * g for v in n]
        k, j, i = np.meshgrid(np.arange(N[2]), np.arange(N[1]), np.arange(N[0]), indexing="ij")
        lev = [(origin[b][d] + (c - g)) % DOMAIN[d] for d, c in enumerate((i, j, k))]
        exp[bx.offset + i + N[0] * (j + N[1] * k)] = lev[0] + DOMAIN[0] * (lev[1] + DOMAIN[1] * lev[2])
    return exp


DOMAIN = (20, 12, 9)
CASES = {
    # name: cuts, shift, reconstruction (ghost width 2, 3, 4)
    "aligned_ppm": (((0, 5, 13, 20), (0, 4, 12), (0, 3, 9)), (0, 0, 0), "ppm"),
    "straddling_plm": (((0, 7, 20), (0, 6, 12), (0, 9)), (3, 5, 7), "plm"),
    # boxes thinner than the ghost width: ghosts from boxes further away
    "thin_boxes_ppm": (((0, 2, 3, 11, 20), (0, 1, 12), (0, 2, 5, 9)), (1, 11, 2), "ppm"),
    "one_box_pc": (((0, 20), (0, 12), (0, 9)), (4, 0, 8), "pc"),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("fofc", [False, True])
def test_exchange_table_fills_every_ghost_once(case, fofc):
    cuts, shift, recon = CASES[case]
    P = ctmhd.make_params(recon=recon, fofc=fofc, emf="q26")
    ng = ctmhd.required_ghosts(P)
    boxes, origin, total = _level(DOMAIN, cuts, shift, ng)
    d = ctmhd.parse_plan(ctmhd.level_plan(P, boxes, origin, DOMAIN))
    assert d["level"] == 1 and d["nbox"] == len(boxes) and d["xbox"][-1] == len(d["xblk"])
    out, writes = _apply(d, boxes, origin, total)
    exp = _expected(boxes, origin, total)
    inside = exp >= 0
    assert np.array_equal(out[inside], exp[inside])
    ghost = inside & (writes > 0)
    assert (writes[inside] <= 1).all()
    assert ghost.sum() == sum(ctmhd.lib().ctmhd_box_elems(b) - int(np.prod(b.n)) for b in boxes)


@pytest.mark.parametrize("fofc", [False, True])
@pytest.mark.parametrize("emf", ["q26", "b25a"])
def test_level_phases(fofc, emf):
    cuts, shift, _ = CASES["aligned_ppm"]
    P = ctmhd.make_params(recon="ppm", fofc=fofc, emf=emf)
    boxes, origin, _ = _level(DOMAIN, cuts, shift, 4)
    d = ctmhd.parse_plan(ctmhd.level_plan(P, boxes, origin, DOMAIN))
    kinds, xarg = d["kind"], d["xarg"]
    lo, hi = d["range"][0]
    assert kinds[lo:hi] == [PH_XCHG, PH_DT] and xarg[lo] == XG_CUR
    lo, hi = d["range"][1]
    expect = []
    for st in range(2):
        tgt = XG_HALF if st == 0 else XG_NEXT
        expect += [(PH_P, 0)] if emf != "q26" else []
        expect += [(PH_FIRST, 0)] if emf != "q26" else []  # PPM: first steps stored
        expect += [(PH_F, 0), (PH_E, 0), (PH_U, 0), (PH_XCHG, tgt | (XG_FLAGS if fofc else 0))]
        if fofc:
            expect += [(PH_O, 0), (PH_X, 0), (PH_XCHG, tgt | XG_IF_FIXUP)]
    assert list(zip(kinds[lo:hi], xarg[lo:hi])) == expect
    # first-order pass of a level: positions 0..n per axis
    per = 256 * d["strips"]
    for p in range(lo, hi):
        if kinds[p] != PH_O:
            continue
        for k in range(len(boxes)):
            b = boxes[d["order"][k]]
            cnt = d["prefix"][p][k + 1] - d["prefix"][p][k]
            assert cnt == -(-((b.n[0] + 1) * (b.n[1] + 1) * (b.n[2] + 1)) // per)


def test_batched_plan_has_no_exchange():
    cuts, shift, _ = CASES["aligned_ppm"]
    P = ctmhd.make_params(recon="ppm", fofc=True)
    boxes, _, _ = _level(DOMAIN, cuts, shift, 4)
    d = ctmhd.parse_plan(ctmhd.batch_plan(P, boxes))
    assert d["level"] == 0 and PH_XCHG not in d["kind"]


@pytest.mark.parametrize("what", ["overlap", "gap", "dx", "origin", "too_big"])
def test_bad_levels_are_refused(what):
    P = ctmhd.make_params(recon="plm")
    cuts, shift, _ = CASES["aligned_ppm"]
    boxes, origin, _ = _level(DOMAIN, cuts, shift, 3)
    domain = list(DOMAIN)
    if what == "overlap":
        origin = origin.copy()
        origin[1] = origin[0]            # two boxes on the same cells, one box's cells missing
    elif what == "gap":
        domain[0] += 1                   # one column of the domain covered by no box
    elif what == "dx":
        boxes[2] = ctmhd.make_box(list(boxes[2].n), 3, (0.2, 0.1, 0.1), boxes[2].offset)
    elif what == "origin":
        origin = origin.copy()
        origin[0][0] = DOMAIN[0]
    else:
        domain = [4, 12, 9]
    with pytest.raises(ctmhd.CtmhdError):
        ctmhd.level_plan(P, boxes, origin, domain)


def _step_level_rc(P, boxes, origin, domain, plan=b"\0" * 16):
    """ctmhd_step_level with placeholder device pointers that are never
    dereferenced: every case below fails validation on the host first."""
    import ctypes
    L = ctmhd.lib()
    arr = (ctmhd.Box * len(boxes))(*boxes)
    d = 256
    c5 = ctmhd._PTR5(*([d] * 5))
    c3 = ctmhd._PTR3(*([d] * 3))
    return L.ctmhd_step_level(ctypes.byref(P), len(boxes), arr, ctmhd._i32(origin, 3 * len(boxes)),
                              ctmhd._i32(domain, 3), plan, c5, c3, 1, None, None, None, None, 0,
                              None)


@pytest.mark.parametrize("what", ["gap", "overlap", "null_plan", "persistent", "force_flags"])
def test_step_level_validates_on_the_host(what):
    cuts, shift, _ = CASES["aligned_ppm"]
    P = ctmhd.make_params(recon="plm")
    boxes, origin, _ = _level(DOMAIN, cuts, shift, 3)
    domain, plan = list(DOMAIN), b"\0" * 16
    if what == "gap":
        domain[2] += 2
    elif what == "overlap":
        origin = origin.copy()
        origin[3] = origin[4]
    elif what == "null_plan":
        plan = None
    elif what == "persistent":
        P.tile = ctmhd.make_tile(persistent=True)
    else:
        P.force_flags = 256
    rc = _step_level_rc(P, boxes, origin, domain, plan)
    assert rc == (-2 if what == "persistent" else -1), (what, rc)
    assert ctmhd.lib().ctmhd_last_error() != b""
