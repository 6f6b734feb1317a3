"""Host-side emulation of the index arithmetic of the preconditioner network's kernels
(paper_1307_5824_amd/csrc/pcnet.hip) over every launch shape the library makes from the
arguments it accepts (batches, grids 32..128, N <= 8 res): each global, LDS and per-thread array
index is computed the way the kernel computes it and checked against the size of what it
indexes.  Runs on the CPU; no kernel is launched."""
import numpy as np
import pytest

CH = 32
NB_MAX = 65536   # nblk() cap of the grid-stride launches


def nblk(n, t=256):
    return min((n + t - 1) // t, NB_MAX)


def wrap(i, g):
    return np.bitwise_and(i, g - 1)


def vox(a, b, c, g):
    return (wrap(a, g) * g + wrap(b, g)) * g + wrap(c, g)


# the index maps are the same for every batch (b only offsets by whole grids) and every power-of-two
# grid; these shapes cover a batch boundary and each grid size the tests and the bench launch
SHAPES = [(1, 32), (3, 32), (2, 64), (1, 128)]


@pytest.mark.parametrize("B,g", SHAPES)
def test_conv_mfma_indices(B, g):
    """k_conv_mfma: one wavefront per (batch, v1, v2, 32-voxel segment), 4 per block of 256."""
    segs = g // 32
    rows = B * g * g * segs
    blocks = (rows + 3) // 4
    GV = g ** 3
    # every wave that passes the row check; lanes l in [0, 64)
    row = np.arange(blocks * 4)
    row = row[row < rows]
    seg, r2 = row % segs, row // segs
    b, v1, v2 = r2 // (g * g), (r2 // g) % g, r2 % g
    s0 = 32 * seg
    lane = np.arange(64)
    i, kb = lane & 31, lane >> 5
    for tap in range(27):
        for sgn in (1, -1):
            da, db, dc = sgn * (tap // 9 - 1), sgn * ((tap // 3) % 3 - 1), sgn * (tap % 3 - 1)
            src = vox(v1[:, None] + da, v2[:, None] + db, s0[:, None] + i[None] + dc, g)
            for c0 in (0, 16):
                xi = (b[:, None] * GV + src) * CH + c0 + 8 * kb[None]
                assert xi.min() >= 0 and xi.max() + 7 < B * GV * CH
                lds = ((tap * CH + i) * CH + c0 + 8 * kb) // 8
                assert lds.min() >= 0 and lds.max() < 27 * CH * CH // 8
    t = np.arange(16)
    vi = 8 * (t[None] // 4) + 4 * kb[:, None] + (t[None] % 4)            # (lane, t)
    assert vi.max() < 32
    o = ((b[:, None, None] * GV + (v1[:, None, None] * g + v2[:, None, None]) * g + s0[:, None, None] + vi[None])
         * CH + (lane[None, :, None] & 31))
    assert o.min() >= 0 and o.max() < B * GV * CH


@pytest.mark.parametrize("B,g", SHAPES)
def test_vector_layer_indices(B, g):
    """k_conv_first, k_conv_last, k_conv_last_bwd, k_symmetrise: grid-stride over B g^3 voxels;
    k_wgrad / k_wgrad_last: (chunks, 27) blocks over 256-voxel chunks."""
    GV = g ** 3
    n = B * GV
    i = np.arange(n)
    bb, v = i // GV, i % GV
    v1, v2, v3 = v // (g * g), (v // g) % g, v % g
    for t in range(27):
        for sgn in (1, -1):
            nb = bb * GV + vox(v1 + sgn * (t // 9 - 1), v2 + sgn * ((t // 3) % 3 - 1), v3 + sgn * (t % 3 - 1), g)
            assert nb.min() >= 0 and nb.max() < n
            assert nb.max() * CH + CH - 1 < n * CH
    flip = bb * GV + (wrap(g - v1, g) * g + wrap(g - v2, g)) * g + wrap(g - v3, g)
    assert flip.min() >= 0 and flip.max() < n
    chunks = (n + 255) // 256
    assert chunks * 256 >= n and 27 <= 65535 and chunks < 2 ** 31
    # k_wgrad<CH>: 1024 threads (co, ci); k_wgrad<1>: 32; k_wgrad_last: ci + 8 parts
    assert CH * CH <= 1024 and (CH * CH - 1) // CH < CH


@pytest.mark.parametrize("B,g", SHAPES)
def test_wgrad_mfma_indices(B, g):
    """k_wgrad_mfma: 9 wavefronts per block, about 512 blocks over runs of rows (b, v1, v2, segment);
    staging chunks of gz (threads < 128) and of each wavefront's neighbour row with its halo
    (34 voxels, chunks l + 64 q < 136), operand gathers from LDS, atomics into dW and db."""
    GV = g ** 3
    segs = g // 32
    rows = B * g * g * segs
    rpb = (rows + 511) // 512
    wblocks = (rows + rpb - 1) // rpb
    assert wblocks <= 512 and wblocks * rpb >= rows and (wblocks - 1) * rpb < rows
    row = np.arange(rows)                       # every row some block visits (r0 <= row < r1)
    seg, r2 = row % segs, row // segs
    b, v1, v2 = r2 // (g * g), (r2 // g) % g, r2 % g
    s0 = 32 * seg
    tid = np.arange(128)
    v, c8 = tid // (CH // 8), tid % (CH // 8)
    gzi = (b[:, None] * GV + (v1[:, None] * g + v2[:, None]) * g + s0[:, None] + v[None]) * CH + 8 * c8[None]
    assert gzi.min() >= 0 and gzi.max() + 7 < B * GV * CH
    assert tid.max() < 32 * CH // 8
    lane = np.arange(64)
    for wave in range(9):
        da, db = wave // 3 - 1, wave % 3 - 1
        for q in range(3):
            c = lane + 64 * q
            c = c[c < 34 * CH // 8]
            p, cc = c // (CH // 8), c % (CH // 8)
            src = vox(v1[:, None] + da, v2[:, None] + db, s0[:, None] - 1 + p[None], g)
            xi = (b[:, None] * GV + src) * CH + 8 * cc[None]
            assert xi.min() >= 0 and xi.max() + 7 < B * GV * CH
            assert c.max() < 34 * CH // 8                       # xs[wave] chunk
        i, kb = lane & 31, lane >> 5
        for kk in range(2):
            k0 = 16 * kk + 8 * kb
            ga = (k0[:, None] + np.arange(8)[None]) * CH + i[:, None]
            assert ga.min() >= 0 and ga.max() < 32 * CH         # gz row in LDS
            xa = (k0[:, None] + np.arange(10)[None]) * CH + i[:, None]
            assert xa.min() >= 0 and xa.max() < 34 * CH         # halo row in LDS
        t = np.arange(16)
        co = 8 * (t[None] // 4) + 4 * kb[:, None] + t[None] % 4
        d = (co * CH + i[:, None]) * 27 + 3 * wave
        assert d.min() >= 0 and d.max() + 2 < CH * CH * 27
        # the three taps of the wave are the kernel's tap = 9 a + 3 b + c with (a, b) = (da, db) + 1
        assert {3 * wave + c for c in range(3)} == {9 * (da + 1) + 3 * (db + 1) + c for c in range(3)}


def _interp(i, N, g):
    u = np.float32(i - N // 2) * (np.float32(g) / np.float32(N))
    fl = np.floor(u)
    lo = fl.astype(np.int64)
    return wrap(lo + g // 2, g), wrap(lo + 1 + g // 2, g), u - fl


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256])
@pytest.mark.parametrize("g", [32, 64, 128, 256])
def test_upsample_and_adjoint_indices(N, g):
    """upsample_at reads the coarse grid at its interpolation corners; k_upsample_adj gathers,
    per axis, the fine indices within one coarse cell into private arrays of 24 entries."""
    if N > 8 * g:
        pytest.skip("rejected on the host: N <= 8 res")
    i = np.arange(N)
    c0, c1, t = _interp(i, N, g)
    assert c0.min() >= 0 and c1.max() < g and np.all((t >= 0) & (t < 1))
    rad = N // g + 1
    for uc in range(g):
        centre = int(np.trunc((uc - g // 2) * N / g)) + N // 2   # C integer division truncates
        q = np.arange(centre - rad, centre + rad + 1)
        assert q.size <= 24
        qi = ((q % N) + N) % N
        a0, a1, tt = _interp(qi, N, g)
        w = np.where(a0 == uc, 1 - tt, 0) + np.where(a1 == uc, tt, 0)
        # every fine index whose interpolation reads uc with a nonzero weight lies in the window
        allw = np.where(c0 == uc, 1 - t, 0) + np.where(c1 == uc, t, 0)
        assert set(i[allw != 0].tolist()) <= set(qi[w != 0].tolist())
        assert np.count_nonzero(w) <= 24


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256])
def test_loss_kernel_partials(N):
    """k_loss_grad and k_kap_sums write min(nblk(N^3), 1024) partials (twice for Kaporin) into
    4096 doubles; the host reads them back into 4096 pinned doubles."""
    lblocks = min(nblk(N ** 3), 1024)
    assert 2 * lblocks <= 4096
