"""CPU models of the index logic that keeps the kernels' memory accesses in
bounds, each checked against brute force.  They restate, step for step, the
enumeration the device code performs (fold images of the box-mode spreading,
anchor pieces of the clipped spreading, the FFT slot walks and their
reciprocal quotients, the real-space pair enumeration), so that the limits
the planner enforces (at most kMaxFoldImages box images per direction, at
most kMaxPieces anchor pieces, at most kMaxClipRanges particle ranges) are
shown to cover every geometry it accepts.
"""
import itertools
import math

import numpy as np
import pytest

K_MAX_FOLD_IMAGES = 8   # se_internal.h
K_MAX_PIECES = 4
K_MAX_CLIP_RANGES = 512
K_SB = 4
K_FFT_BLOCK = 256


# --- box-mode spreading: tile boxes that meet a tile (fold pass) ------------

def box_of(G, T, nt, P, per, t, d):
    """Tile u = t + d wrapped into [0, nt) with the image shift, and the box
    origin u T + shift - (P/2 - 1); None past a free boundary."""
    u, shift = t + d, 0
    while u < 0:
        if not per:
            return None
        u += nt
        shift -= G
    while u >= nt:
        if not per:
            return None
        u -= nt
        shift += G
    return u, u * T + shift - (P // 2 - 1)


def fold_images(G, T, P, per, t):
    """The kernel's enumeration for tile t (one direction): offsets scanned
    over +-reach, boxes kept if they meet [x0, x0 + ext)."""
    nt = (G + T - 1) // T
    RX = T + P - 1
    emin = min(T, G - (nt - 1) * T) if per else T
    reach = 2 + (T + P) // max(emin, 1)
    x0, ext = t * T, min(T, G - t * T)
    out = []
    for d in range(-reach, reach + 1):
        b = box_of(G, T, nt, P, per, t, d)
        if b is None:
            continue
        u, o = b
        if o < x0 + ext and o + RX > x0:
            out.append((u, o))
    return out


def fold_brute(G, T, P, per, t):
    """Every (tile, image) box that meets tile t: tiles u with origin
    u T + k G - (P/2 - 1) for all images k (one image if not periodic)."""
    nt = (G + T - 1) // T
    RX = T + P - 1
    x0, ext = t * T, min(T, G - t * T)
    ks = range(-(RX // G) - 3, RX // G + 4) if per else (0,)
    out = []
    for u in range(nt):
        for k in ks:
            o = u * T + k * G - (P // 2 - 1)
            if o < x0 + ext and o + RX > x0:
                out.append((u, o))
    return out


def test_fold_enumeration_matches_brute_force():
    """For every periodic or free direction of up to 70 grid points, tile
    edges 4-32 (multiples of 4) and even P up to 16: the kernel's offset scan
    finds exactly the boxes that meet the tile, each once; the planner's
    count (the same scan, maximum over tiles) therefore bounds what the fold
    kernel needs, and the plan is refused above kMaxFoldImages.  For the
    tile edges the planner picks by default (4-16), no geometry needs more
    than 7 images."""
    most_default = 0
    for P in range(2, 17, 2):
        for T in range(4, 33, 4):
            for G in range(max(P, 4), 71):
                for per in (True, False):
                    if not per and G < P:
                        continue
                    nt = (G + T - 1) // T
                    counts = []
                    for t in range(nt):
                        k = fold_images(G, T, P, per, t)
                        b = fold_brute(G, T, P, per, t)
                        assert sorted(k) == sorted(b) and len(set(k)) == len(k), (P, T, G, per, t)
                        counts.append(len(k))
                    if T <= 16:
                        most_default = max(most_default, max(counts))
    assert most_default <= K_MAX_FOLD_IMAGES - 1


# --- clipped spreading: anchor pieces of a tile ------------------------------

def floor_div(a, b):
    return a // b   # Python floors for b > 0, as the device helper does


def anchor_pieces(G, per, lo, hi):
    """The kernel's pieces (sub-bin segment, image shift) of anchor cells
    [lo, hi] (unwrapped); at most K_MAX_PIECES."""
    if not per:
        lo, hi = max(lo, 0), min(hi, G - 1)
        return [(lo // K_SB, hi // K_SB, 0, lo, hi)] if lo <= hi else []
    out = []
    k = floor_div(lo, G)
    while k <= floor_div(hi, G) and len(out) < K_MAX_PIECES:
        a, e = max(lo - k * G, 0), min(hi - k * G, G - 1)
        if a <= e:
            out.append((a // K_SB, e // K_SB, k * G, a, e))
        k += 1
    return out


def clip_dim_max(G, T, P, per, pieces_only):
    """The planner's bound: largest sub-bin count (or piece count) of any
    tile, or a value above every limit when a tile needs more pieces."""
    nt = (G + T - 1) // T
    h = P // 2
    most = 0
    for t in range(nt):
        o, e = t * T, min(T, G - t * T)
        lo, hi = o - h, o + e - 1 + h - 1
        if not per:
            lo, hi = max(lo, 0), min(hi, G - 1)
            cnt, npc = (hi // K_SB - lo // K_SB + 1, 1) if lo <= hi else (0, 0)
        else:
            cnt = npc = 0
            for k in range(floor_div(lo, G), floor_div(hi, G) + 1):
                a, b = max(lo - k * G, 0), min(hi - k * G, G - 1)
                if a <= b:
                    cnt += b // K_SB - a // K_SB + 1
                    npc += 1
        if npc > K_MAX_PIECES:
            return 1 << 28
        most = max(most, npc if pieces_only else cnt)
    return most


def test_clipped_anchor_pieces_match_brute_force():
    """The anchors whose stencil c - P/2 + 1 .. c + P/2 meets a tile are the
    cells [o - P/2, o + e - 1 + P/2 - 1]; the kernel's pieces cover exactly
    these cells (as wrapped cell and image shift), each once, whenever the
    planner accepts the geometry, and the planner's range bound covers every
    tile's ranges."""
    for P in range(2, 17, 2):
        for T in range(4, 33, 4):
            for G in range(max(P, 4), 71):
                for per in (True, False):
                    bound = clip_dim_max(G, T, P, per, False)
                    if bound >= 1 << 28:
                        continue        # refused by the planner (boxes and fold instead)
                    nt = (G + T - 1) // T
                    for t in range(nt):
                        o, e = t * T, min(T, G - t * T)
                        lo, hi = o - P // 2, o + e - 1 + P // 2 - 1
                        pcs = anchor_pieces(G, per, lo, hi)
                        assert len(pcs) <= K_MAX_PIECES
                        got = sorted((c, sh) for (_, _, sh, a, b) in pcs for c in range(a, b + 1))
                        want = sorted(((c % G, c - c % G) if per else (c, 0)) for c in range(lo, hi + 1)
                                      if per or 0 <= c < G)
                        assert got == want, (P, T, G, per, t)
                        # every such anchor's stencil reaches the tile
                        for c, sh in got:
                            s0 = c + sh - P // 2 + 1
                            assert s0 < o + e and s0 + P > o
                        nsub = sum(s1 - s0 + 1 for (s0, s1, _, _, _) in pcs)
                        assert nsub <= bound


def test_clip_range_bound_is_an_upper_bound():
    """Ranges per tile = z sub-bins x y sub-bins x x pieces, bounded by the
    product of the per-direction maxima the planner checks against
    kMaxClipRanges."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        P = int(rng.choice(range(2, 17, 2)))
        T = [int(v) for v in rng.choice(range(4, 33, 4), 3)]
        G = [int(v) for v in rng.integers(max(P, 4), 71, 3)]
        per = [bool(v) for v in rng.integers(0, 2, 3)]
        bz, by, bx = (clip_dim_max(G[2], T[2], P, per[2], False), clip_dim_max(G[1], T[1], P, per[1], False),
                      clip_dim_max(G[0], T[0], P, per[0], True))
        if max(bz, by, bx) >= 1 << 28:
            continue
        for tz in range((G[2] + T[2] - 1) // T[2]):
            for ty in range((G[1] + T[1] - 1) // T[1]):
                for tx in range((G[0] + T[0] - 1) // T[0]):
                    n = 1
                    for d, (t, sub) in enumerate(((tx, False), (ty, True), (tz, True))):
                        o, e = t * T[d], min(T[d], G[d] - t * T[d])
                        pcs = anchor_pieces(G[d], per[d], o - P // 2, o + e - 1 + P // 2 - 1)
                        n *= sum(s1 - s0 + 1 for (s0, s1, _, _, _) in pcs) if sub else len(pcs)
                    assert n <= bz * by * bx


# --- FFT pencil blocks: slot walks by additions ------------------------------

def _rcp(d):
    return np.float32(1.0) / np.float32(d)


def test_reciprocal_quotient_is_exact():
    """fdiv(a, rcp(d)) = trunc((a + 1/2) rcp(d)) in FP32 equals a div d for
    all dividends a < 2^13 (kFftCap) and divisors d <= 2^13, also when the
    hardware reciprocal is off by two ulps either way."""
    a = np.arange(8192, dtype=np.float32) + np.float32(0.5)
    ai = np.arange(8192)
    for d in range(1, 8193):
        r0 = _rcp(d)
        for r in (r0, np.nextafter(np.nextafter(r0, 0, dtype=np.float32), 0, dtype=np.float32),
                  np.nextafter(np.nextafter(r0, 1, dtype=np.float32), 1, dtype=np.float32)):
            q = (a * np.float32(r)).astype(np.int64)
            assert np.array_equal(q, ai // d), d


def slot_walk(n, B, gs0, gst, lt, lp, TF, steps):
    """The kernel's per-thread walk over slots tid, tid + 256, ...: (t, p,
    global offset, LDS index) after each step, for all 256 threads at once.
    The fast index (t if TF, else p) runs to lim (n, else B); a step moves the
    slow index by q and the fast one by r, wrapping the fast one."""
    tid = np.arange(K_FFT_BLOCK)
    lim = n if TF else B
    q = K_FFT_BLOCK // lim
    r = K_FFT_BLOCK - q * lim
    slow, fast = tid // lim, tid % lim
    if TF:
        p, t = slow, fast
        dg, dgw = r * gst + q * gs0, gs0 - n * gst
        dl, dlw = r * lt + q * lp, lp - n * lt
    else:
        t, p = slow, fast
        dg, dgw = r * gs0 + q * gst, gst - B * gs0
        dl, dlw = r * lp + q * lt, lt - B * lp
    g = p * gs0 + t * gst
    l = t * lt + p * lp
    out = []
    for _ in range(steps):
        out.append((t.copy(), p.copy(), g.copy(), l.copy()))
        fast, slow = (t, p) if TF else (p, t)
        fast, slow, g, l = fast + r, slow + q, g + dg, l + dl
        w = fast >= lim
        fast = np.where(w, fast - lim, fast)
        slow = np.where(w, slow + 1, slow)
        g = np.where(w, g + dgw, g)
        l = np.where(w, l + dlw, l)
        t, p = (fast, slow) if TF else (slow, fast)
    return out


def _smooth_lengths(limit):
    out = []
    for n in range(2, limit + 1):
        m = n
        for f in (2, 3, 5, 7):
            while m % f == 0:
                m //= f
        if m == 1:
            out.append(n)
    return out


def test_slot_walk_equals_direct_indexing():
    """Walking slots by additions gives, at every step, the slot's direct
    coordinates: pencil-major (p = e div n, t = e mod n) when the transform
    direction is contiguous, sample-major (t = e div B, p = e mod B)
    otherwise, and the matching global offsets and LDS indices, for every
    7-smooth length with block pencil counts B = 1-64 and the even B up to
    128 of the paired real passes (n B <= 8192, or 16384 for even B > 1),
    every B for n <= 512 and a spread of them above."""
    rng = np.random.default_rng(1)
    all_b = list(range(1, 65)) + list(range(66, 129, 2))
    for n in _smooth_lengths(8192):
        Bs = all_b if n <= 512 else [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 24, 32, 64, 128]
        for B in Bs:
            if n * B > (16384 if B % 2 == 0 else 8192):
                continue
            gs0, gst = int(rng.integers(1, 5000)), int(rng.integers(1, 5000))
            lt, lp = B + 1, 1
            steps = (n * B + K_FFT_BLOCK - 1) // K_FFT_BLOCK
            for TF in (True, False):
                walk = slot_walk(n, B, gs0, gst, lt, lp, TF, steps)
                for k, (t, p, g, l) in enumerate(walk):
                    e = np.arange(K_FFT_BLOCK) + k * K_FFT_BLOCK
                    tt, pp = (e % n, e // n) if TF else (e // B, e % B)
                    assert np.array_equal(t, tt) and np.array_equal(p, pp), (n, B, TF, k)
                    assert np.array_equal(g, pp * gs0 + tt * gst) and np.array_equal(l, tt * lt + pp * lp)


# --- real space: the pair enumeration of the cell list ------------------------

def rs_span(h, rc):
    s = max(1, math.ceil(rc / h))
    while s > 1 and (s - 1) * h >= rc:
        s -= 1
    while s * h < rc:
        s += 1
    return s


def rs_cells(L, rc, n_max, k=2):
    by_n = max(1, int(math.floor(float(np.cbrt(max(1, n_max))) + 1e-9)))
    c = int(max(1.0, min(math.floor(k * L / rc), by_n, 160)))
    return c, rs_span(L / c, rc)


def rs_cells_box(Ls, rc, n_max, k=2):
    per = (max(1, n_max) / (Ls[0] * Ls[1] * Ls[2])) ** (1 / 3)
    c = [int(max(1.0, min(math.floor(k * Ld / rc), max(1, math.floor(Ld * per + 1e-9)), 160))) for Ld in Ls]
    return c, [rs_span(Ls[d] / c[d], rc) for d in range(3)]


def rs_candidates(D, c, s, Ls, rc, cells, t):
    """The kernel's candidates for target t: (neighbour, image vector) in the
    order it visits them; c, s and Ls per direction."""
    h = [Ls[d] / c[d] for d in range(3)]
    ix, iy, iz = cells[t]
    out = []
    by_cell = {}
    for j, cc in enumerate(cells):
        by_cell.setdefault(tuple(cc), []).append(j)
    for dz in range(-s[2], s[2] + 1):
        uz = iz + dz
        if D < 3 and not 0 <= uz < c[2]:
            continue
        qz = uz // c[2]
        gz = max(0, abs(dz) - 1) * h[2]
        for dy in range(-s[1], s[1] + 1):
            uy = iy + dy
            if D < 2 and not 0 <= uy < c[1]:
                continue
            qy = uy // c[1]
            gy = max(0, abs(dy) - 1) * h[1]
            rem = rc * rc - gz * gz - gy * gy
            if rem <= 0.0:
                continue
            dm = s[0]
            while dm > 1 and ((dm - 1) * h[0]) ** 2 >= rem:
                dm -= 1
            xa, xb = ix - dm, ix + dm
            if D < 1:
                xa, xb = max(xa, 0), min(xb, c[0] - 1)
            for qx in range(xa // c[0], xb // c[0] + 1):
                lo, hi = max(xa, qx * c[0]) - qx * c[0], min(xb, qx * c[0] + c[0] - 1) - qx * c[0]
                for cx in range(lo, hi + 1):
                    for j in by_cell.get((cx, uy - qy * c[1], uz - qz * c[2]), []):
                        if (qx, qy, qz) == (0, 0, 0) and j == t:
                            continue
                        out.append((j, (qx, qy, qz)))
    return out


def _check_enumeration(D, Ls, rc, n, seed, ks=(1, 2, 3), cells_of=None):
    rng = np.random.default_rng(seed)
    Ls = np.asarray(Ls, dtype=float)
    x = rng.random((n, 3)) * Ls
    for k in ks:
        c, s = cells_of(k)
        c, s = np.asarray(c), np.asarray(s)
        h = Ls / c
        cells = np.minimum((x / h).astype(int), c - 1)
        K = [math.ceil(rc / Ls[d]) + 1 for d in range(3)]
        for t in range(0, n, 7):
            cand = rs_candidates(D, c, s, Ls, rc, [tuple(v) for v in cells], t)
            assert len(cand) == len(set(cand))
            got = set()
            box2 = (rc * (1.0 + 1e-5) + 1e-5 * h.max()) ** 2
            for j, (qx, qy, qz) in cand:
                shift = np.array([qx, qy, qz]) * Ls
                p = x[j] + shift - cells[t] * h   # in the target cell's frame
                e = np.maximum(np.maximum(-p, p - h), 0.0)
                if float(e @ e) >= box2:
                    continue
                if np.linalg.norm(x[t] - (x[j] + shift)) < rc:
                    got.add((j, (qx, qy, qz)))
            # brute force over every charge and image vector
            img = np.array(list(itertools.product(*[range(-K[d], K[d] + 1) if D > d else (0,)
                                                    for d in range(3)])))
            # the distance evaluated as the kernel's candidate test does, so
            # that a pair at rc within rounding falls on the same side
            r = np.linalg.norm(x[t][None, None, :] - (x[:, None, :] + (img * Ls)[None, :, :]), axis=2)
            want = {(int(j), tuple(int(v) for v in img[m])) for j, m in zip(*np.nonzero(r < rc))
                    if not (j == t and not img[m].any())}
            assert got == want, (D, tuple(Ls), rc, k, t)


@pytest.mark.parametrize("D", [3, 2, 1, 0])
@pytest.mark.parametrize("rc_over_L", [0.11, 0.3, 0.55, 1.1, 1.6])
def test_real_space_enumeration_visits_each_pair_once(D, rc_over_L):
    """Every pair within rc (periodic images included, the target itself at
    zero shift excluded) is visited exactly once, for spans s = 1-3 and
    cutoffs beyond the box, also after the kernel drops the candidates that
    lie rc or more from the target cell's box."""
    L, n = 1.0, 90
    rc = rc_over_L * L

    def cells_of(k):
        c, s = rs_cells(L, rc, n, k)
        return [c] * 3, [s] * 3

    _check_enumeration(D, (L, L, L), rc, n, int(100 * rc_over_L) + D, cells_of=cells_of)


@pytest.mark.parametrize("D", [3, 2])
@pytest.mark.parametrize("Ls", [(1.0, 1.5, 0.5), (0.6, 1.0, 1.9), (2.0, 0.35, 1.0)])
@pytest.mark.parametrize("rc", [0.12, 0.3, 0.7, 1.3])
def test_real_space_enumeration_in_rectangular_boxes(D, Ls, rc):
    """The same in rectangular boxes, triply periodic or with z free, with
    cells, spans and cell sides per direction (spans differing between
    directions, cutoffs beyond the short side)."""
    n = 90

    def cells_of(k):
        return rs_cells_box(Ls, rc, n, k)

    _check_enumeration(D, Ls, rc, n, int(1000 * rc + 10 * Ls[1]) + D, cells_of=cells_of)
