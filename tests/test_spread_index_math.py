"""Host-side emulation of the index arithmetic of the fixed-point gridding accumulation
(paper_1307_5824_amd/csrc/spread.hip, k_spread with FX): the footprint lane map (rows split
among the 16-lane groups of an 8-byte LDS access), the 64-bit tile indices of every add, the
staged-point record, and the lane roles of the one read that carries the FQ points' window
words and axis-0 weights to the readlane broadcasts.  Computed the way the kernel computes them
and checked against the sizes of what they index, for every tile and window width the library
launches: the kernel's tile 13 and the A*b tile 12, one component per launch (a one-plane tile),
widths 4..8; and the FP32 plane test and candidate rows of both gridding kernels (spread and
forward projector) against every point of random views at N = 256.  Runs on the CPU; no kernel
is launched."""
import itertools

import numpy as np
import pytest

SP_QCAP, FQ, NTH = 1024, 4, 512
LDS_CU = 160 * 1024


def place_rows(r, W, rp, G, grp):
    if r == W:
        return True
    cap = 64 // G
    for g in range(G):
        n = sum(1 for q in range(r) if grp[q] == g)
        if (n + 1) * W > cap:
            continue
        ok = all((q * rp + i) % cap != (r * rp + j) % cap
                 for q in range(r) if grp[q] == g for i in range(W) for j in range(W))
        if not ok:
            continue
        grp[r] = g
        if place_rows(r + 1, W, rp, G, grp):
            return True
    return False


def row_groups(rp, W, G):
    grp = [0] * 8
    if not place_rows(0, W, rp, G, grp):
        return -1
    return sum(grp[r] << (2 * r) for r in range(W))


def row_pitch(PT, W, G):
    for rp in range(PT, PT + 32):
        if row_groups(rp, W, G) >= 0:
            return rp
    return PT


def lane_map(W, groups, G=4):
    """(j2, j3, act) of every lane, as the kernel derives them."""
    out = []
    for lane in range(64):
        j2 = j3 = 0
        act = False
        if groups >= 0:
            g, idx = lane // (64 // G), lane % (64 // G)
            rank = idx // W
            seen = 0
            for r in range(W):
                if (groups >> (2 * r)) & 3 != g:
                    continue
                if seen == rank:
                    j2, j3, act = r, idx - rank * W, True
                seen += 1
        else:
            act = lane < W * W
            jl = lane if act else 0
            j2, j3 = jl // W, jl - (jl // W) * W
        out.append((j2, j3, act))
    return out


# (tile, width, complex data): the complex data is spread one component per launch into a
# one-plane tile of signed terms, so both cases index one plane
CASES = [(13, W, False) for W in range(4, 9)] + [(12, W, True) for W in range(4, 9)]


@pytest.mark.parametrize("T,W,cplx", CASES)
def test_footprint_lanes_and_tile_indices(T, W, cplx):
    PT = T + W
    RP = row_pitch(PT, W, 4)
    PP = PT * RP
    NV = 1
    groups = row_groups(RP, W, 4)
    lanes = lane_map(W, groups)
    cells = [(j2, j3) for j2, j3, act in lanes if act]
    # every footprint cell has exactly one lane
    assert sorted(cells) == [(a, b) for a in range(W) for b in range(W)]
    if groups >= 0:
        # within each group of 16 lanes the active cells fall in distinct 8-byte banks
        for g in range(4):
            offs = [(j2 * RP + j3) % 16 for j2, j3, act in lanes[16 * g:16 * g + 16] if act]
            assert len(offs) == len(set(offs))
    # every add of every point lands in the tile: window starts are clamped to [0, PT - W]
    size = NV * PT * PP
    for l0, l1, l2 in itertools.product((0, 1, PT - W - 1, PT - W), repeat=3):
        for j2, j3, act in lanes:
            if not act:
                continue
            cb = l0 * PP + (l1 + j2) * RP + l2 + j3
            for r in range(W):
                idx = cb + r * PP
                assert 0 <= idx < size
    # the tile's flush visits each cell once: li = l0 PP + l1 RP + l2 over PT^3 cells, distinct
    li = {(a * PP + b * RP + c) for a in range(PT) for b in range(PT) for c in range(PT)}
    assert len(li) == PT ** 3 and max(li) < PT * PP


def staging_batch(T, W, cplx):
    """The kernel's batch size and record stride: the most points, in whole rounds of FQ per
    wavefront, with one staging item (point, axis) per thread and the workgroup's LDS (the rest
    of it counted as the kernel counts it) within 80 KB up to W = 7, 160 KB at W = 8."""
    PT = T + W
    RP = row_pitch(PT, W, 4)
    qcap = SP_QCAP + 256 if cplx else SP_QCAP - 32  # the queue: 1280 entries for A*b, 992 for Ker
    fixed = PT * PT * RP * 8 + NTH * 4 * (3 if cplx else 1) + (264 * 4 if cplx else 0) + qcap * 4 + 512
    pstr = 3 * W
    per = pstr * 4 + 4
    budget = (160 if W >= 8 else 80) * 1024
    rnd = FQ * NTH // 64
    pb = NTH // 3 // rnd * rnd
    while pb > rnd and fixed + pb * per > budget:
        pb -= rnd
    return pb, pstr, fixed + pb * per


@pytest.mark.parametrize("T,W,cplx", CASES)
def test_staged_record_and_uniform_read(T, W, cplx):
    SP_PB, PSTR, lds = staging_batch(T, W, cplx)
    assert SP_PB % (FQ * NTH // 64) == 0 and 3 * SP_PB <= NTH
    # staging: item (point p, axis d) writes weights at p PSTR + W d + j and byte d of pt_lo[p]
    for p, d, j in itertools.product(range(SP_PB), range(3), range(W)):
        assert p * PSTR + W * d + j < SP_PB * PSTR and W * d + j < PSTR
        assert 4 * p + d < 4 * SP_PB
    # the accumulation's own reads: axis-1 and axis-2 weights of its footprint cell
    for p, j in itertools.product((0, SP_PB - 1), range(W)):
        assert p * PSTR + W + j < SP_PB * PSTR and p * PSTR + 2 * W + j < SP_PB * PSTR
    # the uniform read: roles of the lanes and the lanes the readlanes take
    assert FQ * 8 + FQ <= 64
    for nb in sorted({1, 2, 7, 8, 9, 33, 95, 96, SP_PB - 1, SP_PB}):
        for wv in range(NTH // 64):
            for p0 in range(wv, nb, FQ * (NTH // 64)):
                pq = [min(p0 + q * (NTH // 64), nb - 1) for q in range(FQ)]
                for lane in range(64):
                    if lane < 32:
                        uq = lane >> 3
                    elif lane < 32 + FQ:
                        uq = lane - 32
                    else:
                        uq = ((lane - 32 - FQ) >> 1) % FQ
                    pl = pq[uq]
                    assert 0 <= pl < nb
                    if lane < 32:
                        assert pl * PSTR + (lane & 7) < SP_PB * PSTR
                    else:
                        assert pl < SP_PB
                # readlane sources: weight r of point q, window word of q
                for q in range(FQ):
                    for r in range(W):
                        assert (8 * q + r) >> 3 == q and (8 * q + r) & 7 == r
                    assert 32 + q - 32 == q
    # the A*b staging reads the disk's row starts from LDS (N + 1 entries loaded, 264 declared)
    # at k1 + N/2 for the half disk's rows 0 <= k1 <= N/2
    for N in (8, 16, 32, 64, 128, 256):
        assert max(k1 + N // 2 for k1 in range(N // 2 + 1)) <= N < 264
    # LDS of one workgroup: the 64-bit tile, the staged points, the queue, the view slots (and the
    # slots' views and groups and the row starts for complex data); two workgroups share a CU up
    # to width 7.  At the widths the library runs by default (7) the batch holds 128 points for
    # the kernel's tile and 160 for the A*b tile.
    wgs = 1 if W >= 8 else 2
    assert wgs * lds <= LDS_CU
    if W == 7:
        assert SP_PB == (160 if cplx else 128)


def test_fixed_point_sums_are_exact_and_order_free():
    """The tile adds integer terms below 2^31 in 64-bit cells: any order gives the same sum, and
    up to 2^32 terms cannot overflow, so the flush sees the exact sum of the rounded terms."""
    rng = np.random.default_rng(5)
    terms = rng.integers(-(2 ** 31) + 1, 2 ** 31, 10000, dtype=np.int64)
    s1 = int(np.sum(terms))
    s2 = int(np.sum(rng.permutation(terms)))
    assert s1 == s2 == sum(int(t) for t in terms)
    assert (2 ** 31) * (2 ** 32) <= 2 ** 63


@pytest.mark.parametrize("T,L", [(13, 1024), (12, 512)])
def test_normal_box_culling_never_drops_a_view(T, L):
    """The spread (and the forward projector, tile 12 on the 2N grid) skips a block of 512 views
    when the box of their (hemisphere-folded) normals gives no |n . c| within 0.5 T max|n|_1 +
    3e-3 of the tile's centre c.  Emulated with the kernel's expressions (FP32 normals, FP64
    products): whenever some view of a block passes the per-view plane test, the block test
    passes too; and the test does prune."""
    rng = np.random.default_rng(11 + T)
    M = 4096
    # a concentrated cluster and uniform directions, as the workloads' view distributions
    n = rng.standard_normal((M, 3))
    n[: M // 2] = n[: M // 2] * 0.2 + np.array([0.3, 0.5, 0.8])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n = n.astype(np.float32)
    ax = np.argmax(np.abs(n), axis=1)
    sg = np.where(n[np.arange(M), ax] < 0, -1.0, 1.0).astype(np.float32)
    nf = n * sg[:, None]
    u = n[np.arange(M), (ax + 1) % 3] / n[np.arange(M), ax]
    v = n[np.arange(M), (ax + 2) % 3] / n[np.arange(M), ax]
    qu = np.clip((u + 1.0) * 511.5, 0, 1023).astype(np.int64)
    qv = np.clip((v + 1.0) * 511.5, 0, 1023).astype(np.int64)
    mort = np.zeros(M, dtype=np.int64)
    for b in range(10):
        mort |= ((qu >> b) & 1) << (2 * b) | ((qv >> b) & 1) << (2 * b + 1)
    order = np.argsort((ax.astype(np.int64) << 20) | mort, kind="stable")
    ns = nf[order]
    skipped = 0
    for t in range(200):
        tc = (rng.integers(0, L // T, 3) * T + 0.5 * T - 0.5 * L).astype(np.float64)
        for bk in range(M // 512):
            blk = ns[bk * 512:(bk + 1) * 512].astype(np.float64)
            per_view = np.abs(blk @ tc) <= 0.5 * T * np.abs(blk).sum(axis=1) + 2e-3
            lo, hi = blk.min(axis=0).astype(np.float32), blk.max(axis=0).astype(np.float32)
            l1 = np.float32(np.abs(blk).sum(axis=1).max() * (1 + 1e-6))
            p, q = tc * lo.astype(np.float64), tc * hi.astype(np.float64)
            dmin, dmax = np.minimum(p, q).sum(), np.maximum(p, q).sum()
            lim = 0.5 * T * float(l1) + 3e-3
            live = dmin <= lim and dmax >= -lim
            assert live or not per_view.any()
            skipped += not live
    assert skipped > 0


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))[None, :]


@pytest.mark.parametrize("T,kind", [(13, "spread"), (12, "spread"), (12, "project")])
def test_plane_test_and_candidate_rows_cover_every_point(T, kind):
    """Both gridding kernels keep a view for a tile when the FP32 plane test passes, and then
    enumerate S candidate rows k1 from a start computed in FP32 from the tile's centre c:
    u1 = <c, c1> / s, the spread from ceil(u1 - rk - 1e-3) with S = floor(2 rk + 2e-3) + 2, the
    forward projector from ceil(u1 - rk) - 1 with S = floor(2 rk) + 3, rk = (0.866 T + 1e-3) / s.
    Every half-disk point (|k| <= N/2) of a view at N = 256 (grid 2N, s = 2) must have its
    clamped cell's tile pass the plane test and its k1 among that tile's candidate rows."""
    rng = np.random.default_rng(17 + T)
    N = 256
    L, s = 2 * N, 2.0
    f32 = np.float32
    kk = np.arange(-N // 2, N // 2 + 1)
    k1, k2 = np.meshgrid(kk, kk, indexing="ij")
    disk = 4 * (k1 * k1 + k2 * k2) <= N * N
    k1, k2 = k1[disk], k2[disk]
    rk = (f32(T) * f32(0.8660254) + f32(1e-3)) / f32(s)
    if kind == "spread":
        S = int(np.floor(f32(2) * rk + f32(2e-3))) + 2
    else:
        S = int(np.floor(f32(2) * rk)) + 3
    for _ in range(24):
        R = _rotation(rng)
        c1, c2 = R[:, 0], R[:, 1]
        nv = np.cross(c1, c2).astype(f32)
        tau = s * (k2[:, None] * c2[None, :] + k1[:, None] * c1[None, :]) + 0.5 * L
        tt = np.clip(np.floor(tau), 0, L - 1).astype(np.int64) // T
        tc = (tt.astype(f32) * f32(T) + f32(0.5 * T) - f32(0.5 * L)).astype(f32)
        dist = np.abs(tc[:, 0] * nv[0] + tc[:, 1] * nv[1] + tc[:, 2] * nv[2])
        lim = f32(0.5) * f32(T) * (np.abs(nv[0]) + np.abs(nv[1]) + np.abs(nv[2])) + f32(2e-3)
        assert np.all(dist <= lim)
        c1f = c1.astype(f32)
        dot = tc[:, 0] * c1f[0] + tc[:, 1] * c1f[1] + tc[:, 2] * c1f[2]
        if kind == "spread":
            u1 = dot * (f32(1) / f32(s))
            start = np.ceil(u1 - rk - f32(1e-3)).astype(np.int64)
        else:
            u1 = dot / f32(s)
            start = np.ceil(u1 - rk).astype(np.int64) - 1
        assert np.all(k1 >= start) and np.all(k1 < start + S)


def test_live_block_chunks_visit_every_live_block_once():
    """The culling tests up to 512 blocks of views at a time into a bit mask, then one thread
    hands out the live blocks in chunks of VPT = 8 (scanning 32-bit words from a cursor, skipping
    empty words).  Emulated as the kernel does it: the chunks list every set bit once, in order."""
    rng = np.random.default_rng(23)
    VPT = 8
    for density in (0.0, 0.01, 0.2, 0.9, 1.0):
        for nblk in (1, 31, 32, 33, 300, 512):
            bits = (rng.random(nblk) < density)
            mask = [0] * 16
            for b in np.flatnonzero(bits).tolist():
                mask[b >> 5] |= 1 << (b & 31)
            seen, cur = [], 0
            while True:
                n, chunk = 0, []
                while n < VPT and cur < 512:
                    w = mask[cur >> 5] & ((0xFFFFFFFF << (cur & 31)) & 0xFFFFFFFF)
                    if w == 0:
                        cur = (cur | 31) + 1
                        continue
                    b = (cur & ~31) + ((w & -w).bit_length() - 1)
                    chunk.append(b)
                    n += 1
                    cur = b + 1
                if not chunk:
                    break
                assert len(chunk) <= VPT
                seen += chunk
            assert seen == np.flatnonzero(bits).tolist()
