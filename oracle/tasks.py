"""Plain fp64 reference math of the task kernels (test infrastructure).

Every function takes float32 arrays (the in-memory type of the workloads),
computes in float64 and rounds its outputs once to float32, unless noted.
The paper describes the benchmarks only in prose (Sec. V-B); where it fixes
no formula the textbook definition named in each docstring is used, and the
readings are listed in the design notes.
"""

import math

import numpy as np
from scipy import special

F32 = np.float32
F64 = np.float64


# --------------------------------------------------------------------------
# VEC (Sec. V-B, "Vector Squares"): square two vectors, sum their difference.
# --------------------------------------------------------------------------
def vec_square(x):
    """x_i <- x_i * x_i, one correctly rounded float32 product.

    The float64 product of two float32 values is exact (48 significant bits),
    so rounding it once to float32 is the IEEE single-precision product.
    """
    xd = np.asarray(x, dtype=F32).astype(F64)
    return (xd * xd).astype(F32)


def vec_sum_diff(x, y):
    """r = sum_i (x_i - y_i), exact sum (math.fsum) rounded to float32.

    float32 - float32 is exact in float64 for the value ranges used here, and
    fsum returns the correctly rounded float64 sum, so the only rounding that
    matters is the final one to float32.
    """
    d = np.asarray(x, dtype=F32).astype(F64) - np.asarray(y, dtype=F32).astype(F64)
    return F32(math.fsum(d.tolist()))


# --------------------------------------------------------------------------
# B&S (Sec. V-B, "Black & Scholes" for European call options; the paper uses
# double precision).  Textbook closed form.
# --------------------------------------------------------------------------
def norm_cdf(z):
    """Standard normal CDF Phi(z) = erfc(-z / sqrt(2)) / 2 in float64."""
    return 0.5 * special.erfc(-np.asarray(z, dtype=F64) / math.sqrt(2.0))


def bs_call(S, K, r, sigma, T):
    """European call price C = S Phi(d1) - K e^{-rT} Phi(d2), float64 -> float32.

    d1 = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt(T)),  d2 = d1 - sigma sqrt(T).
    """
    s = np.asarray(S, dtype=F32).astype(F64)
    vol_t = sigma * math.sqrt(T)
    d1 = (np.log(s / K) + (r + 0.5 * sigma * sigma) * T) / vol_t
    d2 = d1 - vol_t
    c = s * norm_cdf(d1) - K * math.exp(-r * T) * norm_cdf(d2)
    return c.astype(F32)


# --------------------------------------------------------------------------
# IMG (Sec. V-B, "Image Processing": a sharpened picture combined with copies
# blurred at low and medium frequencies, to sharpen edges and soften the
# rest).  Gaussian blur, Sobel edge magnitude, min/max normalisation and an
# unsharp-mask combine; replicate (clamp-to-edge) borders.
# --------------------------------------------------------------------------
def gauss_weights(ksize):
    """1-D Gaussian weights w_i ~ exp(-i^2 / (2 s^2)), s = ksize/6, sum 1."""
    if ksize < 1 or ksize % 2 == 0:
        raise ValueError("ksize must be odd and positive")
    sigma = ksize / 6.0
    rad = (ksize - 1) // 2
    i = np.arange(-rad, rad + 1, dtype=F64)
    w = np.exp(-(i * i) / (2.0 * sigma * sigma))
    return w / w.sum()


def _shifted(img, dy, dx):
    """img[clamp(y+dy), clamp(x+dx)] for every pixel (replicate border)."""
    h, w = img.shape
    ys = np.clip(np.arange(h) + dy, 0, h - 1)
    xs = np.clip(np.arange(w) + dx, 0, w - 1)
    return img[ys][:, xs]


def gauss_blur(img, ksize):
    """2-D Gaussian blur: out = sum_{i,j} w_i w_j img[y+i, x+j], float64 -> float32.

    Written as the direct 2-D correlation (no separable factoring) so it can
    be checked by eye.
    """
    a = np.asarray(img, dtype=F32).astype(F64)
    w = gauss_weights(ksize)
    rad = (ksize - 1) // 2
    out = np.zeros_like(a)
    for i in range(-rad, rad + 1):
        for j in range(-rad, rad + 1):
            out += (w[i + rad] * w[j + rad]) * _shifted(a, i, j)
    return out.astype(F32)


SOBEL_X = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]])
SOBEL_Y = SOBEL_X.T


def sobel(img):
    """Sobel gradient magnitude sqrt(gx^2 + gy^2), float64 -> float32.

    gx = correlation with [[-1,0,1],[-2,0,2],[-1,0,1]], gy with its transpose.
    """
    a = np.asarray(img, dtype=F32).astype(F64)
    gx = np.zeros_like(a)
    gy = np.zeros_like(a)
    for i in range(-1, 2):
        for j in range(-1, 2):
            s = _shifted(a, i, j)
            gx += SOBEL_X[i + 1, j + 1] * s
            gy += SOBEL_Y[i + 1, j + 1] * s
    return np.sqrt(gx * gx + gy * gy).astype(F32)


def minmax(img):
    """(max, min) of a float32 array, exact."""
    a = np.asarray(img, dtype=F32)
    return F32(a.max()), F32(a.min())


def normalise(img, mx, mn):
    """(S - mn) / (mx - mn) in float64 -> float32; all zeros when mx == mn."""
    a = np.asarray(img, dtype=F32).astype(F64)
    mx = F64(F32(mx))
    mn = F64(F32(mn))
    if mx == mn:
        return np.zeros(a.shape, dtype=F32)
    return ((a - mn) / (mx - mn)).astype(F32)


def unsharp_combine(img, b3, b7, b15, n3, n7, n15):
    """Combine: E = (N3+N7+N15)/3, sharp = 2 img - B3 (unsharp mask, amount 1),
    soft = (B7 + B15)/2, out = clamp(E sharp + (1 - E) soft, 0, 1).
    float64 -> float32.
    """
    f = [np.asarray(v, dtype=F32).astype(F64) for v in (img, b3, b7, b15, n3, n7, n15)]
    img, b3, b7, b15, n3, n7, n15 = f
    e = (n3 + n7 + n15) / 3.0
    sharp = 2.0 * img - b3
    soft = 0.5 * (b7 + b15)
    out = e * sharp + (1.0 - e) * soft
    return np.clip(out, 0.0, 1.0).astype(F32)


# --------------------------------------------------------------------------
# HITS (Sec. V-B: repeated SpMV on a matrix and its transpose).  Kleinberg's
# hubs and authorities, in the form where both products read the previous
# iterate, each vector normalised by its L2 norm.
# --------------------------------------------------------------------------
def spmv(row_ptr, col, val, x):
    """y_r = sum_{k in row r} val_k x_{col_k}; float64 sums in index order
    (np.bincount accumulates sequentially), rounded to float32."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    nrows = row_ptr.size - 1
    rows = np.repeat(np.arange(nrows), np.diff(row_ptr))
    prod = np.asarray(val, dtype=F32).astype(F64) * np.asarray(x, dtype=F32).astype(F64)[np.asarray(col)]
    y = np.bincount(rows, weights=prod, minlength=nrows)
    return y.astype(F32)


def sumsq(v):
    """s = sum_i v_i^2 as a float64 scalar (exact sum, correctly rounded)."""
    vd = np.asarray(v, dtype=F32).astype(F64)
    return F64(math.fsum((vd * vd).tolist()))


def scale_l2(t, s):
    """v_i = t_i / sqrt(s) in float64, rounded to float32."""
    td = np.asarray(t, dtype=F32).astype(F64)
    return (td / math.sqrt(F64(s))).astype(F32)


def hits(a_ptr, a_col, a_val, at_ptr, at_col, at_val, iters):
    """HITS iterations: auth <- A^T hub, hub <- A auth (both from the previous
    iterate), each L2-normalised.  Returns (auth, hub) as float32."""
    n = len(a_ptr) - 1
    auth = np.ones(n, dtype=F32)
    hub = np.ones(n, dtype=F32)
    for _ in range(iters):
        at = spmv(at_ptr, at_col, at_val, hub)
        ht = spmv(a_ptr, a_col, a_val, auth)
        auth = scale_l2(at, sumsq(at))
        hub = scale_l2(ht, sumsq(ht))
    return auth, hub


# --------------------------------------------------------------------------
# ML ensemble (Sec. V-B, "Machine Learning Ensemble"): a categorical naive
# Bayes classifier and a ridge classifier on standardised features score the
# same input rows; each row of scores is softmax-normalised, the two
# probability rows are averaged and the class with the largest average is
# the prediction.  X is an (n, F) float32 matrix whose entries are category
# codes 0..V-1 (read as integers by naive Bayes, as numbers by ridge).
# --------------------------------------------------------------------------
def softmax_rows(S):
    """P[r, c] = exp(S[r, c] - m_r) / sum_c' exp(S[r, c'] - m_r) with
    m_r = max_c S[r, c] (the shift leaves P unchanged and keeps exp finite);
    float64 in, float64 out."""
    S = np.asarray(S, dtype=F64)
    E = np.exp(S - S.max(axis=1, keepdims=True))
    return E / E.sum(axis=1, keepdims=True)


def nb_log_joint(X, log_theta, log_prior):
    """Joint log-likelihood of categorical naive Bayes, float64:
    J[r, c] = log pi_c + sum_f log theta[c, f, X[r, f]].

    log_theta has shape (C, F, V): log P(feature f = v | class c);
    log_prior has shape (C,): log P(class c)."""
    codes = np.asarray(X, dtype=F32).astype(np.int64)
    lt = np.asarray(log_theta, dtype=F32).astype(F64)
    C, F, _ = lt.shape
    J = np.tile(np.asarray(log_prior, dtype=F32).astype(F64), (codes.shape[0], 1))
    for f in range(F):
        J += lt[:, f, codes[:, f]].T
    return J


def nb_predict_proba(X, log_theta, log_prior):
    """Class posteriors of categorical naive Bayes: softmax of the joint
    log-likelihood over classes, rounded to float32, shape (n, C)."""
    return softmax_rows(nb_log_joint(X, log_theta, log_prior)).astype(F32)


def ridge_scores(X, mean, scale, W, b):
    """Decision scores of a linear (ridge) classifier on standardised
    features, float64: S = ((X - mean) / scale) W^T + b, W of shape (C, F)."""
    Z = (np.asarray(X, dtype=F32).astype(F64) - np.asarray(mean, dtype=F32).astype(F64)) \
        / np.asarray(scale, dtype=F32).astype(F64)
    return Z @ np.asarray(W, dtype=F32).astype(F64).T + np.asarray(b, dtype=F32).astype(F64)


def ridge_predict_proba(X, mean, scale, W, b):
    """Softmax of the ridge scores over classes, rounded to float32."""
    return softmax_rows(ridge_scores(X, mean, scale, W, b)).astype(F32)


def ensemble_argmax(p_nb, p_rr):
    """Average of the two probability rows and the predicted class.

    avg = (p_nb + p_rr) / 2 is exact in float64 for float32 inputs; the label
    is the first index of the largest float64 average (lowest class index on
    ties), the average is returned rounded to float32."""
    avg = (np.asarray(p_nb, dtype=F32).astype(F64) + np.asarray(p_rr, dtype=F32).astype(F64)) / 2.0
    return avg.astype(F32), np.argmax(avg, axis=1).astype(np.int32)


# --------------------------------------------------------------------------
# DL (Sec. V-B, "Deep Learning"): a convolutional network projects two input
# images to low-dimensional embeddings and a dense layer combines them.
# Layers (the paper names only the structure): 3x3 convolution with zero
# padding (cross-correlation, as in deep-learning frameworks), bias, ReLU and
# 2x2 max pooling; a dense embedding layer; a dense combining layer with a
# sigmoid.  Tensors are channel-major (C, H, W) float32.
# --------------------------------------------------------------------------
def conv3x3_relu_pool(x, w, b):
    """y[o] = maxpool2x2(relu(b[o] + sum_c corr3x3(x[c], w[o, c]))), float64 in
    registers, rounded once to float32.  x: (C_in, H, W) with H, W even;
    w: (C_out, C_in, 3, 3); b: (C_out,).  Returns (C_out, H/2, W/2)."""
    x = np.asarray(x, dtype=F32).astype(F64)
    w = np.asarray(w, dtype=F32).astype(F64)
    b = np.asarray(b, dtype=F32).astype(F64)
    cin, h, wd = x.shape
    cout = w.shape[0]
    xp = np.zeros((cin, h + 2, wd + 2))
    xp[:, 1:h + 1, 1:wd + 1] = x
    z = np.empty((cout, h, wd))
    for o in range(cout):
        acc = np.full((h, wd), b[o])
        for c in range(cin):
            for dy in range(3):
                for dx in range(3):
                    acc += w[o, c, dy, dx] * xp[c, dy:dy + h, dx:dx + wd]
        z[o] = acc
    z = np.maximum(z, 0.0)
    pooled = z.reshape(cout, h // 2, 2, wd // 2, 2).max(axis=(2, 4))
    return pooled.astype(F32)


def dense(x, w, b):
    """y = W x + b for a flattened input, float64, rounded to float32;
    W: (M, N), x: (N,), b: (M,)."""
    x = np.asarray(x, dtype=F32).astype(F64).ravel()
    w = np.asarray(w, dtype=F32).astype(F64)
    return (w @ x + np.asarray(b, dtype=F32).astype(F64)).astype(F32)


def siamese_combine(e1, e2, w, b):
    """p = sigmoid(w . [e1; e2] + b) as a float32 scalar (float64 inside)."""
    z = np.concatenate([np.asarray(e1, dtype=F32).astype(F64), np.asarray(e2, dtype=F32).astype(F64)])
    s = float(np.dot(np.asarray(w, dtype=F32).astype(F64), z)) + float(np.float32(b))
    return F32(1.0 / (1.0 + math.exp(-s)))
