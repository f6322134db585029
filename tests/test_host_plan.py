"""Host-side logic of the native library, no GPU: exported symbols, grid
detection, and the tree / skeleton plan against the CPU reference."""
import os
import re

import numpy as np
import pytest

from oracle import rskel
from paper_1303_5466_amd import rsd, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = rsd.load()
    hdr = open(os.path.join(ROOT, "include", "rsd.h")).read()
    names = set(re.findall(r"\b(rsd_[a-z_0-9]+)\s*\(", hdr))
    assert "rsd_build_factor" in names and "rsd_solve" in names and "rsd_free" in names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(rsd.EXPORTS) <= names


@pytest.mark.parametrize("nx,ny,seed", [(16, 16, 0), (37, 37, 1), (40, 24, 2), (3, 5, 3)])
def test_detect_grid_shuffled(nx, ny, seed):
    pts = W.grid_points(nx, ny)
    sp, perm = W.shuffled(pts, seed)
    gx, gy, h, pm = rsd.detect_grid(sp)
    assert (gx, gy) == (nx, ny)
    assert h == pytest.approx(1.0 / max(nx, ny))
    assert np.array_equal(sp[pm], pts)


def test_detect_grid_rejects_non_grids():
    pts = W.grid_points(8)
    with pytest.raises(rsd.RsdError) as e:
        rsd.detect_grid(pts[:-1])
    assert e.value.status == rsd.RSD_ENOTGRID
    dup = pts.copy()
    dup[5] = dup[6]
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(dup)
    jit = pts.copy()
    jit[10, 0] += 0.3 / 8
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(jit)
    stretched = pts.copy()
    stretched[:, 1] *= 2.0
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(stretched)
    nan = pts.copy()
    nan[3, 1] = np.nan
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(nan)
    # uneven columns with a matching point count: x in {0, 1, 3, 4}
    uneven = np.array([[x, y] for x in (0.0, 1.0, 3.0, 4.0) for y in range(4)], dtype=float)
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(uneven)
    # one point moved half a spacing off its line
    half = pts.copy()
    half[20, 1] += 0.5 / 8
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(half)
    with pytest.raises(rsd.RsdError):
        rsd.detect_grid(pts[:1])


def test_detect_grid_offset_and_line_grids():
    # origin anywhere, spacing from the point set; single rows and columns
    pts = W.grid_points(12, 9) * 3.0 - np.array([7.5, -2.25])
    gx, gy, h, pm = rsd.detect_grid(pts[::-1].copy())
    assert (gx, gy) == (12, 9) and h == pytest.approx(3.0 / 12)
    assert np.array_equal(pts[::-1][pm], pts)
    line = np.array([[0.25, 0.5 + 0.125 * j] for j in range(7)])
    gx, gy, h, pm = rsd.detect_grid(line[::-1].copy())
    assert (gx, gy) == (1, 7) and h == pytest.approx(0.125)


@pytest.mark.parametrize("nx,ny,leaf,m", [(64, 64, 8, 2), (40, 24, 8, 2), (37, 37, 8, 2),
                                         (32, 32, 8, 3), (16, 16, 8, 1), (8, 8, 8, 2), (20, 7, 4, 2)])
def test_plan_matches_reference_sets(nx, ny, leaf, m):
    """Every box's active, skeleton and residual sets equal the reference's
    (Sec. 3.1 layer rule); the library's order is its own."""
    plan = rsd.Plan(nx, ny, leaf, m)
    root, levels = rskel.index_sets(nx, ny, leaf, m)
    D = len(levels) - 1
    assert plan.n_levels == D + 1
    box = 0
    for t in range(D + 1):
        for b in levels[D - t]:
            info = plan.box_info(box)
            assert (info["x0"], info["y0"], info["ax"], info["ay"]) == (b.x0, b.y0, *b.shape)
            pts = plan.box_points(box)
            k, r = info["k"], info["r"]
            if t == D:
                # the root keeps every active point: second child first, then the first
                assert set(pts.tolist()) == set(b.act.tolist())
            else:
                assert set(pts[:k].tolist()) == set(b.act[b.sk].tolist())
                assert set(pts[k:].tolist()) == set(b.act[b.rs].tolist())
            box += 1
    assert box == plan.n_boxes


@pytest.mark.parametrize("nx,ny,m,step", [(64, 64, 3, 3), (50, 40, 2, 1), (96, 64, 3, 5), (37, 37, 3, 2)])
def test_plan_interface_points_match_reference_sets(nx, ny, m, step):
    """With interface skeleton points (Sec. 5.3) every box's skeleton and
    residual sets still equal the reference's."""
    plan = rsd.Plan(nx, ny, 8, m, interface_step=step)
    root, levels = rskel.index_sets(nx, ny, 8, m, step)
    D = len(levels) - 1
    box = 0
    extra = 0
    for t in range(D + 1):
        for b in levels[D - t]:
            info = plan.box_info(box)
            pts = plan.box_points(box)
            k = info["k"]
            if t < D:
                assert set(pts[:k].tolist()) == set(b.act[b.sk].tolist())
                assert set(pts[k:].tolist()) == set(b.act[b.rs].tolist())
                i, j = b.act[b.sk] // ny, b.act[b.sk] % ny
                d = np.minimum.reduce([i - b.x0, b.x1 - 1 - i, j - b.y0, b.y1 - 1 - j])
                extra += int(np.sum(d >= m))
            box += 1
    assert extra > 0


@pytest.mark.parametrize("ax,ay,m,step", [(32, 16, 3, 3), (64, 32, 2, 4), (16, 16, 3, 1), (40, 20, 3, 6)])
def test_interface_points_rule(ax, ay, m, step):
    """The reference's interface rule on one box cut across x: the extra
    skeleton points lie on the two grid lines beside the cut, mirror
    symmetric about the box's centre lines, consecutive ones step cells
    apart along the cut in each half (at most 2 step across the middle),
    none inside the boundary layers."""
    b = rskel.Box(0, ax, 0, ay, 0)
    c1 = rskel.Box(0, ax // 2, 0, ay, 1)
    c2 = rskel.Box(ax // 2, ax, 0, ay, 1)
    b.children = [c1, c2]
    ii, jj = np.meshgrid(np.arange(ax), np.arange(ay), indexing="ij")
    i, j = ii.ravel(), jj.ravel()
    base = rskel.skeleton_mask(b, i, j, m, 0)
    with_iface = rskel.skeleton_mask(b, i, j, m, step)
    assert np.all(with_iface[base])
    ex = with_iface & ~base
    ei, ej = i[ex], j[ex]
    assert set(ei.tolist()) == {ax // 2 - 1, ax // 2}
    pts = set(zip(ei.tolist(), ej.tolist()))
    assert all((ax - 1 - u, v) in pts and (u, ay - 1 - v) in pts for u, v in pts)
    assert ej.min() >= m and ej.max() <= ay - 1 - m
    for u in (ax // 2 - 1, ax // 2):
        vs = np.sort(ej[ei == u])
        lower = vs[vs <= (ay - 1) / 2]
        assert np.all(np.diff(lower) == step)
        assert np.all(np.diff(vs) <= 2 * step)
        assert len(vs) >= (ay - 2 * m) // step - 1
    # a leaf (no children) gets no interface points
    leaf = rskel.Box(0, ax, 0, ay, 0)
    assert np.array_equal(rskel.skeleton_mask(leaf, i, j, m, step), base)


def test_interface_step_from_wavenumber():
    """floor(2 pi / (k h ppw)) cells for ppw points per wavelength."""
    assert rskel.interface_step(100.0, 1.0 / 128, 4.0) == 2      # 8.04 cells per wavelength
    assert rskel.interface_step(20.0, 1.0 / 256, 4.0) == 20      # 80.4 cells
    assert rskel.interface_step(200.0, 1.0 / 64, 8.0) == 1       # under a cell: one


def test_plan_levels_golden():
    """Per-depth box shapes and sizes stored in tests/golden/levels.txt."""
    path = os.path.join(ROOT, "tests", "golden", "levels.txt")
    cur = None
    expect = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        if tok[0] == "grid":
            cur = tuple(int(x) for x in tok[1:])
            expect[cur] = []
        else:
            expect[cur].append(tuple(int(x) for x in tok))
    for (nx, ny, leaf, m), rows in expect.items():
        plan = rsd.Plan(nx, ny, leaf, m)
        D = plan.n_levels - 1
        got = {}
        for b in range(plan.n_boxes):
            i = plan.box_info(b)
            depth = D - i["level"]
            if depth == 0:
                continue
            key = (depth, i["ax"], i["ay"], i["k"], i["r"])
            got[key] = got.get(key, 0) + 1
        want = {(d, ax, ay, k, r): c for (d, ax, ay, c, k, r, p) in rows if d > 0}
        assert got == want, (nx, ny)


def test_layer_count_reads_tolerance():
    assert rskel.layers_for_tol(1e-10) == 2


@pytest.mark.parametrize("nx,ny", [(64, 64), (50, 50), (75, 75), (37, 24), (40, 24)])
def test_box_symmetry_by_brute_force(nx, ny):
    """The reflection group the interpolation split uses: a mirror reflection
    (along an even side) belongs to it exactly when it maps the box's skeleton
    and residual sets onto themselves (the proxy ring is always symmetric)."""
    P = rsd.Plan(nx, ny, 8, 2)
    groups = []
    for b in range(P.n_boxes):
        info = P.box_info(b)
        if info["r"] == 0 or info["parent"] < 0:
            continue
        ids = P.box_points(b)
        k, ax, ay = info["k"], info["ax"], info["ay"]
        u, v = ids // ny - info["x0"], ids % ny - info["y0"]
        sk, rs = set(zip(u[:k], v[:k])), set(zip(u[k:], v[k:]))

        def closed(flip):
            return {flip(p) for p in sk} == sk and {flip(p) for p in rs} == rs

        expect = 0
        if ax % 2 == 0 and closed(lambda p: (ax - 1 - p[0], p[1])):
            expect |= 1
        if ay % 2 == 0 and closed(lambda p: (p[0], ay - 1 - p[1])):
            expect |= 2
        assert P.box_symmetry(b) == expect, (b, ax, ay)
        groups.append(expect)
    if nx == ny == 64:
        assert set(groups) == {3}            # even halves all the way down
    if nx == ny == 50:
        assert {1, 2} <= set(groups)         # odd halves: one reflection only


def test_batched_entry_points_reject_bad_arguments_on_the_host():
    """Argument errors of the batched calls are reported before any device
    work (these run without a GPU)."""
    import ctypes as C
    lib = rsd.load()
    out = (C.c_void_p * 1)()
    pts = (C.c_void_p * 1)()
    npts = (C.c_int64 * 1)(4)
    kd = rsd.rsd_kernel(rsd.RSD_KERNEL_LAPLACE, 0.0, None)
    assert lib.rsd_build_factor_batched(0, pts, npts, C.byref(kd), None, 1e-10, None, 0, out) == rsd.RSD_EINVAL
    assert lib.rsd_build_factor_batched(1, None, npts, C.byref(kd), None, 1e-10, None, 0, out) == rsd.RSD_EINVAL
    assert "null" in lib.rsd_last_error().decode()
    fs = (C.c_void_p * 2)(None, None)
    ptrs = (C.c_void_p * 2)(None, None)
    assert lib.rsd_solve_batched(0, fs, ptrs, 1, ptrs, None) == rsd.RSD_EINVAL
    assert lib.rsd_solve_batched(2, fs, ptrs, 1, ptrs, None) == rsd.RSD_EINVAL   # null factors


def test_single_calls_reject_bad_arguments_on_the_host():
    """Argument errors of build and solve come back as status codes with a
    message, before any device work; NULL handles are harmless to free."""
    import ctypes as C
    lib = rsd.load()
    kd = rsd.rsd_kernel(rsd.RSD_KERNEL_LAPLACE, 0.0, None)
    pts = np.zeros((4, 2))
    h = C.c_void_p()
    p = pts.ctypes.data
    assert lib.rsd_build_factor(None, 4, C.byref(kd), None, 1e-10, None, C.byref(h)) == rsd.RSD_EINVAL
    assert h.value is None
    assert lib.rsd_build_factor(p, 0, C.byref(kd), None, 1e-10, None, C.byref(h)) == rsd.RSD_EINVAL
    for tol in (0.0, -1.0, float("nan"), float("inf")):
        assert lib.rsd_build_factor(p, 4, C.byref(kd), None, tol, None, C.byref(h)) == rsd.RSD_EINVAL
        assert "tol" in lib.rsd_last_error().decode()
    x = np.zeros(4)
    info = rsd.rsd_solve_info()
    assert lib.rsd_solve(None, x.ctypes.data, 1, x.ctypes.data, C.byref(info)) == rsd.RSD_EINVAL
    lib.rsd_free(None)


@pytest.mark.parametrize("nx,ny", [(64, 64), (50, 50)])
def test_sector_split_reproduces_the_whole_least_squares_solution(nx, ny):
    """The symmetry-adapted split the device uses, checked in NumPy on the
    plan's own sets: for a box type with reflection group G (order 2 or 4),
    solving one least-squares problem per character ab of G, with entries
    sum_g chi_ab(g) K(z - g x) on orbit representatives, and recombining
    T[i, j] = 1/|G| sum_ab chi_ab(g_i) chi_ab(h_j) T_ab[orb_i, orb_j] gives
    the whole problem's solution of K(Z, X_sk) T = K(Z, X_rs)."""
    P = rsd.Plan(nx, ny, 8, 2)
    m = 2
    done = set()
    for b in range(P.n_boxes):
        info = P.box_info(b)
        grp = P.box_symmetry(b)
        if grp == 0 or info["r"] == 0 or info["parent"] < 0:
            continue
        ax, ay, k = info["ax"], info["ay"], info["k"]
        if (ax, ay, grp) in done or max(ax, ay) > 40:
            continue
        done.add((ax, ay, grp))
        ids = P.box_points(b)
        X = np.stack([ids // ny - info["x0"], ids % ny - info["y0"]], axis=1)
        Z = np.array([(u, v) for u in range(-m, ax + m) for v in range(-m, ay + m)
                      if not (0 <= u < ax and 0 <= v < ay)])
        K = lambda zs, xs: 0.5 * np.log(((zs[:, None, :] - xs[None, :, :]) ** 2).sum(-1))
        T = np.linalg.lstsq(K(Z, X[:k]), K(Z, X[k:]), rcond=None)[0]
        refl = [g for g in range(4) if (g & grp) == g]             # the group's elements
        flip = lambda p, g: np.stack([np.where(g & 1, ax - 1 - p[:, 0], p[:, 0]),
                                      np.where(g & 2, ay - 1 - p[:, 1], p[:, 1])], axis=1)
        lower = lambda p: (((p[:, 0] < ax // 2) | (not grp & 1)) & ((p[:, 1] < ay // 2) | (not grp & 2)))

        def orbits(pts):
            rep = pts[lower(pts)]
            g_of = (np.where(bool(grp & 1) & (pts[:, 0] >= ax // 2), 1, 0) +
                    np.where(bool(grp & 2) & (pts[:, 1] >= ay // 2), 2, 0))
            base = flip(pts, g_of)
            index = {tuple(p): i for i, p in enumerate(rep)}
            return rep, np.array([index[tuple(p)] for p in base]), g_of

        zr = Z[lower(Z)]
        skr, sk_orb, sk_g = orbits(X[:k])
        rsr, rs_orb, rs_g = orbits(X[k:])
        parity = np.array([0, 1, 1, 0])                             # popcount parity of 0..3
        chi = lambda ab, g: 1.0 - 2.0 * parity[np.bitwise_and(ab, g)]
        Trec = np.zeros_like(T)
        for ab in refl:                                            # characters, labelled like the elements
            A = sum(chi(ab, g) * K(zr, flip(skr, g)) for g in refl)
            B = sum(chi(ab, g) * K(zr, flip(rsr, g)) for g in refl)
            Tab = np.linalg.lstsq(A, B, rcond=None)[0]
            Trec += (chi(ab, sk_g)[:, None] * chi(ab, rs_g)[None, :]) * Tab[np.ix_(sk_orb, rs_orb)]
        Trec /= len(refl)
        assert np.abs(Trec - T).max() <= 1e-6 * np.abs(T).max(), (ax, ay, grp)
    assert done


def _sides_of_batch(n=6):
    rng = np.random.default_rng(3)
    return [int(s) for s in rng.integers(32, 257, size=n)]


@pytest.mark.parametrize("nx,ny", [(40, 24), (37, 37), (50, 50), (75, 75), (64, 64)]
                         + [(s, s) for s in _sides_of_batch()])
def test_interp_sector_groups(nx, ny):
    """Every interpolation (sector) problem's truncation-scale group is exactly
    its own problem's sectors (Sec. 2.1: the ID truncates at tol |R11| of the
    whole problem): consecutive, inside the list, one owner, the characters of
    the box's reflection group.  The earlier kernel took [i - sec, i - sec + 4),
    which is wrong for every two-sector group; check that such groups exist on
    these grids where expected and that the checker rejects that grouping."""
    plan = rsd.Plan(nx, ny, 8, 2)
    t = plan.interp_groups(split=True)
    n = t.shape[0]
    assert n > 0
    # the group sizes seen by box queries: every split owner's size is the
    # order of some box's reflection group
    orders = {[1, 2, 2, 4][plan.box_symmetry(b)] for b in range(plan.n_boxes)}
    assert set(np.unique(t[:, 3]).tolist()) <= orders | {1}
    two_sector = 0
    i = 0
    while i < n:
        owner, sec, g0, gn, p, k, r = t[i]
        assert g0 == i and gn in (1, 2, 4)
        rows = t[i:i + gn]
        assert (rows[:, 0] == owner).all() and (rows[:, 2] == g0).all() and (rows[:, 3] == gn).all()
        secs = sorted(rows[:, 1].tolist())
        if gn == 1:
            assert secs == [-1]
        elif gn == 2:
            two_sector += 1
            assert secs in ([0, 1], [0, 2])
        else:
            assert secs == [0, 1, 2, 3]
        assert (rows[:, 4:] == rows[0, 4:]).all()
        # the old rule's group for the last sector of a two-sector problem
        if gn == 2:
            last = i + 1
            old_first = last - int(t[last, 1])
            assert (old_first, old_first + 4) != (g0, g0 + gn)
        i += gn
    rsd.check_interp_groups(t)
    # whole problems: one entry each, sizes add up to the split ones
    w = plan.interp_groups(split=False)
    assert (w[:, 1] == -1).all() and (w[:, 3] == 1).all()
    assert (w[:, 2] == np.arange(w.shape[0])).all()
    for o in np.unique(t[:, 0]):
        ts = t[t[:, 0] == o]
        wo = w[w[:, 0] == o]
        assert wo.shape[0] == 1
        assert (ts[:, 4:].sum(axis=0) == wo[0, 4:]).all()
    # which groups have two sectors: odd-half grids have them, 64^2 has none
    if (nx, ny) in [(40, 24), (50, 50), (75, 75)]:
        assert two_sector > 0
    if (nx, ny) == (64, 64):
        assert two_sector == 0
    # the earlier grouping (g0 = i - sec, gn = 4) is rejected wherever a
    # two-sector group exists
    bad = t.copy()
    for j in range(n):
        if bad[j, 1] >= 0:
            bad[j, 2] = j - bad[j, 1]
            bad[j, 3] = 4
    if two_sector:
        with pytest.raises(rsd.RsdError) as e:
            rsd.check_interp_groups(bad)
        assert e.value.status == rsd.RSD_EINVAL
    else:
        rsd.check_interp_groups(bad)


def test_interp_group_checker_rejects_malformed_tables():
    t = rsd.Plan(40, 24, 8, 2).interp_groups(split=True)
    rsd.check_interp_groups(t)
    gi = int(np.nonzero(t[:, 3] > 1)[0][0])
    for mutate in (
        lambda x: x.__setitem__((gi, 2), -1),               # group before the list
        lambda x: x.__setitem__((gi, 3), 3),                # odd group size
        lambda x: x.__setitem__((gi + 1, 1), x[gi, 1]),     # repeated character
        lambda x: x.__setitem__((gi + 1, 0), x[gi, 0] + 1), # two owners in one group
        lambda x: x.__setitem__((gi, 5), x[gi, 5] + 1),     # sectors of unequal size
    ):
        bad = t.copy()
        mutate(bad)
        with pytest.raises(rsd.RsdError):
            rsd.check_interp_groups(bad)
    last = t[-1:].copy()
    last[0, 2], last[0, 3] = 0, 1
    last[0, 1] = -1
    rsd.check_interp_groups(last)
    past = t.copy()
    past[-1, 3] = past[-1, 3] + 1
    with pytest.raises(rsd.RsdError):
        rsd.check_interp_groups(past)


@pytest.mark.parametrize("nx,ny", [(32, 32), (40, 24), (256, 256)])
def test_factor_bytes_estimate_counts_every_block(nx, ny):
    # one (k + r)^2 block per box (float64), plus the interpolation blocks:
    # at least the box blocks, and the float32 form keeps all levels below the
    # root in half the bytes
    p = rsd.Plan(nx, ny, 8, 2)
    boxes = [p.box_info(b) for b in range(p.n_boxes)]
    blocks = sum((b["k"] + b["r"]) ** 2 for b in boxes)
    e64 = rsd.estimate_factor_bytes(nx, ny, 1e-10)
    e32 = rsd.estimate_factor_bytes(nx, ny, 1e-10, precision=rsd.RSD_PREC_FP32_REFINE)
    assert e64 >= 8 * blocks
    top = max(b["level"] for b in boxes)
    root = sum((b["k"] + b["r"]) ** 2 for b in boxes if b["level"] == top)
    assert e32 >= 4 * (blocks - root) + 8 * root and e32 < e64
    with pytest.raises(rsd.RsdError):
        rsd.estimate_factor_bytes(0, 4, 1e-10)


@pytest.mark.parametrize("h,k", [(1 / 64, 20.0), (1 / 128, 20.0), (1 / 512, 20.0), (1 / 32, 60.0)])
def test_self_cell_integral_matches_the_reference(h, k):
    # the library's host quadrature of the Helmholtz cell integral against the
    # CPU reference's (itself pinned against adaptive quadrature); Laplace
    # against the closed form
    from oracle import nystrom
    got = rsd.self_cell_integral(h, rsd.RSD_KERNEL_HELMHOLTZ, k)
    ref = nystrom.self_cell_helmholtz(h, k, nq=60)
    assert abs(got - ref) <= 1e-13 * abs(ref)
    assert rsd.self_cell_integral(h) == pytest.approx(nystrom.self_cell_laplace(h), rel=1e-14)
