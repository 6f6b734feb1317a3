"""FP64 oracle of the learned Fourier-diagonal preconditioner (test infrastructure only).

The preconditioner is P r = F^{-1}(d . F r) on the periodic N^3 grid (a circulant operator,
diagonal in the Fourier basis: section 2.3, eq. circ1), with d > 0 and d(q) = d(-q) so that P
is real, symmetric and positive definite.  d comes from a small network:

  features  f = log(|K^| pooled to G^3 / Ker(0) + lambda_rel)       (G = 32 by default, any power
            of two up to 2N: the network is fully convolutional; K^ = DFT_2N of the circulant
            column, unnormalised: the Fourier multiplier of the embedded product)
  network   o = c4(relu(c3(relu(c2(relu(c1(f)))))))                 (3^3 convolutions,
            circular padding, channels 1 -> C -> C -> C -> 1)
  symmetric s(u) = (o(u) + o(-u)) / 2 on the centred G^3 frequency grid
  diagonal  d(q) = 1 / (t(q) + Ker(0) exp(U s (q))),  U = periodic trilinear interpolation from
            the G^3 grid to the N^3 frequency grid (q -> coarse coordinate q G / N), t the Fourier
            diagonal of A*A + lambda (T. Chan's optimal circulant spectrum).  The network learns a
            floor mu(q) = exp(U s (q)) under the analytic spectrum: mu -> 0 is Chan's 1 / t, and
            a network whose last layer has zero weights gives the constant floor exp(b4).

Objectives:

probe loss  E_z ||P (A*A + lambda) z - z||^2 / E ||z||^2.  With u = (A*A + lambda) z and
            Parseval, for a fixed set of probes it is a per-frequency quadratic in d:
            L(d) = sum_q (d^2 A(q) - 2 d B(q) + C(q)) / sum_q C(q), with A = sum |u^|^2,
            B = sum Re(conj(u^) z^), C = sum |z^|^2 over the probes (u^, z^ the unnormalised
            DFTs; the 1/N^3 of Parseval cancels in the ratio).
Kaporin     the log of Kaporin's condition number of P (A*A + lambda):
            K = (tr(P T) / n)^n / det(P T), n = N^3.  For P diagonal in the Fourier basis,
            tr(P T) = sum_q d(q) t(q) with t(q) = (F T F^*)_{qq} the Fourier diagonal of
            T = A*A + lambda (T. Chan's optimal circulant), and det P = prod d, so
            log K / n = log(mean_q d t) - mean_q log d + const.  It is >= 0 with equality iff
            d is proportional to 1 / t, and invariant to scaling d.
unrolled    the energy-norm error left after k steps of PCG (section 3.3: CG minimises that
            norm over the Krylov space): for a probe z and b = T z, x_k the k-th PCG iterate
            from x0 = 0, L = ||z - x_k||_T^2 / ||z||_T^2.  Its minimiser is not 1 / t: it
            rewards the clustering of the preconditioned spectrum that CG's convergence rests on.

Every gradient here is hand-written and pinned by central finite differences.
"""
import numpy as np

G = 32


# ----------------------------------------------------------------- conv layers --

def conv3d(x, w, b):
    """y[co] = b[co] + sum_ci sum_{a in {-1,0,1}^3} w[co, ci, a + 1] x[ci, i + a] (periodic).
    x (Cin, D, D, D), w (Cout, Cin, 3, 3, 3), b (Cout,)."""
    cout = w.shape[0]
    D = x.shape[1:]
    y = np.empty((cout,) + D)
    for co in range(cout):
        y[co] = b[co]
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                xs = np.roll(x, shift=(-(a - 1), -(bb - 1), -(c - 1)), axis=(1, 2, 3))   # xs[i] = x[i + off]
                y += np.tensordot(w[:, :, a, bb, c], xs, axes=([1], [0]))
    return y


def conv3d_backward(x, w, dy):
    """Gradients of conv3d: dx[ci, i] = sum_co sum_off w[co, ci, off] dy[co, i - off],
    dw[co, ci, off] = sum_i dy[co, i] x[ci, i + off], db[co] = sum_i dy[co, i]."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                off = (a - 1, bb - 1, c - 1)
                xs = np.roll(x, shift=(-off[0], -off[1], -off[2]), axis=(1, 2, 3))
                dw[:, :, a, bb, c] = np.tensordot(dy, xs, axes=([1, 2, 3], [1, 2, 3]))
                t = np.tensordot(w[:, :, a, bb, c], dy, axes=([0], [0]))          # (Cin, D, D, D)
                dx += np.roll(t, shift=off, axis=(1, 2, 3))                        # t[i - off]
    db = dy.sum(axis=(1, 2, 3))
    return dx, dw, db


def init_params(C=32, seed=0, zero_last=True, floor=1.0):
    """He-scaled random weights; with zero_last the last layer's weights start at zero and its
    bias at log(floor), so the untrained network is the constant floor: d = 1 / (t + floor Ker(0))."""
    rng = np.random.default_rng(seed)
    shapes = [(C, 1), (C, C), (C, C), (1, C)]
    params = []
    for i, (co, ci) in enumerate(shapes):
        std = np.sqrt(2.0 / (ci * 27))
        w = rng.standard_normal((co, ci, 3, 3, 3)) * std
        b = np.zeros(co)
        if zero_last and i == 3:
            w[:] = 0.0
            b[:] = np.log(floor)
        params.append((w, b))
    return params


def bf16(a):
    """Round to bfloat16 (round to nearest, ties to even, on the float32 bit pattern), back to float64."""
    x = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    x = (x + 0x7FFF + ((x >> 16) & 1)) >> 16 << 16
    return x.astype(np.uint32).view(np.float32).astype(np.float64)


# layers whose operands the matrix cores read in bfloat16 (the two C -> C layers)
MFMA_LAYERS = (1, 2)


def net_forward(f, params, emulate_bf16=False):
    """o = c4(relu(c3(relu(c2(relu(c1(f))))))); returns o and the cache for backward.
    emulate_bf16 rounds the inputs and weights of the C -> C layers to bfloat16, where the
    GPU's matrix cores read them (the cache keeps the unrounded activations)."""
    x0 = f[None]
    h = x0
    cache = []
    for i, (w, b) in enumerate(params):
        if emulate_bf16 and i in MFMA_LAYERS:
            z = conv3d(bf16(h), bf16(w), b)
        else:
            z = conv3d(h, w, b)
        cache.append((h, z))
        h = np.maximum(z, 0.0) if i < len(params) - 1 else z
    return h[0], cache


def net_backward(do, params, cache, emulate_bf16=False):
    """Gradients of sum(do * o) with respect to the parameters (and the input features).
    emulate_bf16: the C -> C layers' gradients read bfloat16 operands, as the GPU's matrix cores
    do: the data gradient bfloat16 copies of the incoming gradient and of the weights, the weight
    and bias gradients bfloat16 copies of the incoming gradient and of the layer's input (the
    sums themselves are exact here)."""
    grads = [None] * len(params)
    g = do[None]
    for i in range(len(params) - 1, -1, -1):
        h, z = cache[i]
        if i < len(params) - 1:
            g = g * (z > 0)
        if emulate_bf16 and i in MFMA_LAYERS:
            _, dw, db = conv3d_backward(bf16(h), params[i][0], bf16(g))
            dx, _, _ = conv3d_backward(h, bf16(params[i][0]), bf16(g))
        else:
            _, dw, db = conv3d_backward(h, params[i][0], g)
            dx, _, _ = conv3d_backward(h, params[i][0], g)
        grads[i] = (dw, db)
        g = dx
    return grads, g[0]


# ----------------------------------------------------------------- features --

def pool_features(khat_full, ker0, lam_rel, g=G):
    """f = log(mean over (2N/g)^3 blocks of |K^| / Ker(0) + lam_rel), on the centred g^3 grid.
    khat_full: the (2N)^3 spectrum in FFT order."""
    M2 = khat_full.shape[0]
    k = np.fft.fftshift(np.abs(khat_full))
    s = M2 // g
    pooled = k.reshape(g, s, g, s, g, s).mean(axis=(1, 3, 5))
    return np.log(pooled / ker0 + lam_rel)


def symmetrise(o):
    """s(u) = (o(u) + o(-u)) / 2 on the centred coarse grid (index u + G/2)."""
    flipped = np.roll(o[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
    return 0.5 * (o + flipped)


def _interp_axis(N, g=G):
    """Per-axis periodic linear interpolation from g coarse points to N fine points (both centred):
    fine frequency q = i - N/2 sits at coarse coordinate q g / N."""
    q = np.arange(N) - N // 2
    u = q * (g / N)
    lo = np.floor(u).astype(int)
    t = u - lo
    i0 = (lo + g // 2) % g
    i1 = (lo + 1 + g // 2) % g
    return i0, i1, t


def upsample(s, N):
    """U s: periodic trilinear interpolation of the g^3 grid of s onto the N^3 frequency grid."""
    g = s.shape[0]
    out = s
    for ax in range(3):
        i0, i1, t = _interp_axis(N, g)
        a = np.take(out, i0, axis=ax)
        b = np.take(out, i1, axis=ax)
        shape = [1, 1, 1]
        shape[ax] = N
        out = a * (1 - t).reshape(shape) + b * t.reshape(shape)
    return out


def upsample_adjoint(g, N, gc=G):
    """U^T g: the adjoint of upsample from the gc^3 grid (scatter-add of the interpolation weights)."""
    out = g
    for ax in (2, 1, 0):
        i0, i1, t = _interp_axis(N, gc)
        shape = list(out.shape)
        shape[ax] = gc
        acc = np.zeros(shape)
        ws = [1, 1, 1]
        ws[ax] = N
        a = out * (1 - t).reshape(ws)
        b = out * t.reshape(ws)
        for i in range(N):
            sl = [slice(None)] * 3
            sl[ax] = i
            dst0 = [slice(None)] * 3
            dst0[ax] = i0[i]
            dst1 = [slice(None)] * 3
            dst1[ax] = i1[i]
            acc[tuple(dst0)] += a[tuple(sl)]
            acc[tuple(dst1)] += b[tuple(sl)]
        out = acc
    return out


def floor_field(o, N):
    """mu(q) = exp(U sym(o)) on the centred N^3 grid, in units of Ker(0)."""
    return np.exp(upsample(symmetrise(o), N))


def diagonal(o, N, ker0, t):
    """d = 1 / (t + Ker(0) mu) on the centred N^3 grid from the raw network output o."""
    return 1.0 / (t + ker0 * floor_field(o, N))


# ----------------------------------------------------------------- probe loss --

def probe_statistics(apply, N, probes):
    """A, B, C on the centred N^3 grid for the given real probes z (P, N, N, N) and
    u = apply(z): A = sum |u^|^2, B = sum Re(conj(u^) z^), C = sum |z^|^2 (unnormalised DFT)."""
    A = np.zeros((N, N, N))
    B = np.zeros((N, N, N))
    C = np.zeros((N, N, N))
    for z in probes:
        u = apply(z)
        zh = np.fft.fftshift(np.fft.fftn(z))
        uh = np.fft.fftshift(np.fft.fftn(u))
        A += np.abs(uh) ** 2
        B += np.real(np.conj(uh) * zh)
        C += np.abs(zh) ** 2
    return A, B, C


def probe_loss(d, A, B, C):
    """L(d) = sum (d^2 A - 2 d B + C) / sum C = E ||P u - z||^2 / E ||z||^2 (Parseval)."""
    return float(np.sum(d * d * A - 2 * d * B + C) / np.sum(C))


def probe_loss_grad_d(d, A, B, C):
    return (2 * d * A - 2 * B) / np.sum(C)


def kaporin_loss(d, t):
    """log(mean(d t)) - mean(log(d t)): log K(P T) / n with K Kaporin's condition number
    (tr(P T) / n)^n / det(P T), where det T is replaced by prod t (a constant in d).  >= 0 by the
    AM-GM inequality, zero iff d t is constant."""
    dt = d * t
    return float(np.log(np.mean(dt)) - np.mean(np.log(dt)))


def kaporin_grad_logd(d, t):
    """Gradient of kaporin_loss with respect to log d(q)."""
    dt = d * t
    return dt / np.sum(dt) - 1.0 / dt.size


def loss_and_grads(f, params, N, ker0, t, A=None, B=None, C=None, emulate_bf16=False, objective="probe"):
    """Loss of the network on one sample and the gradients of every parameter.  t is the Fourier
    diagonal of A*A + lambda on the centred N^3 grid.  objective "probe": A, B, C are the probe
    statistics; "kaporin": no statistics; "logd": A is the gradient of some loss with respect to
    log d (for instance unrolled_pcg_grad_logd), and the returned loss is None."""
    o, cache = net_forward(f, params, emulate_bf16)
    mu = floor_field(o, N)
    d = 1.0 / (t + ker0 * mu)
    if objective == "kaporin":
        L = kaporin_loss(d, t)
        glogd = kaporin_grad_logd(d, t)
    elif objective == "logd":
        L = None
        glogd = A
    else:
        L = probe_loss(d, A, B, C)
        glogd = probe_loss_grad_d(d, A, B, C) * d
    # log d = -log(t + Ker(0) exp(U s)): d log d / d (U s) = -Ker(0) mu d
    gs = upsample_adjoint(glogd * (-ker0 * mu * d), N, f.shape[0])
    go = symmetrise(gs)                          # symmetrise is self-adjoint
    grads, _ = net_backward(go, params, cache, emulate_bf16)
    return L, grads, d


def flatten_params(params):
    """Host parameter layout of the library: w1 b1 w2 b2 w3 b3 w4 b4."""
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def unflatten_params(vec, C=32):
    shapes = [(C, 1), (C, C), (C, C), (1, C)]
    out, k = [], 0
    for co, ci in shapes:
        nw = co * ci * 27
        w = np.asarray(vec[k:k + nw], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        k += nw
        b = np.asarray(vec[k:k + co], dtype=np.float64)
        k += co
        out.append((w, b))
    return out


def precond_apply(d, r):
    """z = F^{-1}(d . F r), d on the centred grid."""
    return np.fft.ifftn(np.fft.ifftshift(d) * np.fft.fftn(r)).real


# ------------------------------------------------------------ unrolled PCG objective --

def _pcg_steps(apply, d, b, k):
    """k steps of PCG from x0 = 0 on apply(x) = b with P = precond_apply(d, .): the iterate x_k,
    the residuals r_0 .. r_{k-1} and the step lengths alpha_i and ratios beta_i (section 3.3,
    preconditioned)."""
    x = np.zeros_like(b)
    r = b.copy()
    s = precond_apply(d, r)
    p = s.copy()
    rho = float(np.sum(r * s))
    rs, alphas, betas = [], [], []
    for _ in range(k):
        rs.append(r.copy())
        q = apply(p)
        a = rho / float(np.sum(p * q))
        x = x + a * p
        r = r - a * q
        s = precond_apply(d, r)
        rho_new = float(np.sum(r * s))
        bt = rho_new / rho
        p = s + bt * p
        rho = rho_new
        alphas.append(a)
        betas.append(bt)
    return x, rs, alphas, betas


def unrolled_pcg_loss(apply, d, z, k):
    """||z - x_k||_T^2 / ||z||_T^2 with T = apply, b = T z and x_k the k-th PCG iterate."""
    b = apply(z)
    x, _, _, _ = _pcg_steps(apply, d, b, k)
    e = z - x
    return float(np.sum(e * apply(e)) / np.sum(z * b))


def unrolled_pcg_grad_logd(apply, d, z, k):
    """Loss and gradient of unrolled_pcg_loss with respect to log d(q) on the centred grid.

    x_k is the minimiser of the energy-norm error over the preconditioned Krylov space; holding
    the recursion's scalars alpha_i, beta_i fixed, x_k is a fixed polynomial combination of
    (P T)^j P b, so by the envelope theorem the derivative of the minimum equals the derivative
    of that combination.  Reverse pass (adjoints Pbar, Sbar, Rbar of p_i, s_i = P r_i, r_i):
        xbar = -2 T e / ||z||_T^2,
        Pbar_i = alpha_i xbar + beta_i Pbar_{i+1} - alpha_i T Rbar_{i+1},   Sbar_i = Pbar_i,
        Rbar_i = Rbar_{i+1} + P Sbar_i,
        dL/dd(q) += Re(conj(F Sbar_i)(q) (F r_i)(q)) / N^3   (P = F^{-1} diag(d) F, Parseval).
    """
    b = apply(z)
    x, rs, alphas, betas = _pcg_steps(apply, d, b, k)
    e = z - x
    u = apply(e)
    nz = float(np.sum(z * b))
    L = float(np.sum(e * u) / nz)
    xbar = -2.0 * u / nz
    Pbar = np.zeros_like(z)
    Rbar = np.zeros_like(z)
    g = np.zeros(z.shape)
    for i in range(k - 1, -1, -1):
        beta_term = betas[i] * Pbar if i < k - 1 else 0.0
        Pbar = alphas[i] * xbar + beta_term - alphas[i] * apply(Rbar)
        Sbar = Pbar
        g += np.real(np.conj(np.fft.fftn(Sbar)) * np.fft.fftn(rs[i]))
        Rbar = Rbar + precond_apply(d, Sbar)
    return L, np.fft.fftshift(g) / z.size * d
