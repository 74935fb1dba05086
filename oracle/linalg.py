"""Vector kernels, Arnoldi and the two GMRES polynomials of the paper, in FP64.

* The F-point smoother: the GMRES polynomial q of Eq. (gmres_poly) in the
  monomial basis, its coefficients found once per level by Arnoldi on a random
  right-hand side and a small least-squares problem (Sec. 2.2).
* The coarse solver: a high-order GMRES polynomial applied in Newton form with
  the harmonic Ritz values as roots (Sec. 2.3, after Loe & Morgan 2022).

Summation orders are fixed so that setup decisions can be compared bit for bit
with another implementation that follows the same orders: a CSR row sum runs
left to right in ascending column order starting from 0.0, and a dot product
sums the rounded products by a perfect binary tree over the index range padded
with zeros to a power of two (adjacent pairs first).
"""
import math

import numpy as np
import scipy.linalg


# ---------------------------------------------------------------------------
# vector kernels
# ---------------------------------------------------------------------------

def _row_order(A):
    lens = np.diff(A.indptr)
    order = np.argsort(-lens, kind="stable")
    return lens, order, lens[order]


def spmv(A, x):
    """y = A x; each row summed left to right in ascending column order."""
    n = A.shape[0]
    y = np.zeros(n)
    if n == 0 or A.nnz == 0:
        return y
    lens, order, slens = _row_order(A)
    start = A.indptr[:-1].astype(np.int64)
    maxlen = int(slens[0])
    for k in range(maxlen):
        cnt = int(np.searchsorted(-slens, -k, side="left"))   # rows with len > k
        rows = order[:cnt]
        p = start[rows] + k
        y[rows] = y[rows] + A.data[p] * x[A.indices[p]]
    return y


def tree_sum(p):
    """Sum by a perfect binary tree over len(p) padded with zeros to 2^k."""
    n = len(p)
    if n == 0:
        return 0.0
    size = 1 << (n - 1).bit_length()
    t = np.zeros(size)
    t[:n] = p
    while len(t) > 1:
        t = t[0::2] + t[1::2]
    return float(t[0])


def dot(x, y):
    return tree_sum(x * y)


def norm(x):
    return math.sqrt(dot(x, x))


# ---------------------------------------------------------------------------
# Arnoldi with classical Gram-Schmidt applied twice
# ---------------------------------------------------------------------------

BREAKDOWN_TOL = 1e-14


def arnoldi(A, b, m):
    """m steps of Arnoldi on K(A, b).

    Returns (V, H, steps, beta): V the basis vectors, H the (m+1) x m upper
    Hessenberg matrix, steps <= m the number of steps taken (fewer on a happy
    breakdown, when the new direction is below BREAKDOWN_TOL times |A v_j|)
    and beta = |b|.
    """
    beta = norm(b)
    V = [b / beta]
    H = np.zeros((m + 1, m))
    steps = m
    for j in range(m):
        w = spmv(A, V[j])
        w0 = norm(w)
        for _ in range(2):
            h = [dot(V[k], w) for k in range(j + 1)]
            for k in range(j + 1):
                w = w - h[k] * V[k]
            for k in range(j + 1):
                H[k, j] = H[k, j] + h[k]
        hn = norm(w)
        H[j + 1, j] = hn
        if hn <= BREAKDOWN_TOL * w0:
            steps = j + 1
            break
        if j + 1 < m:
            V.append(w / hn)
    return V, H, steps, beta


def givens_lstsq(H, beta):
    """y = argmin |beta e_1 - H y| for an (m+1) x m upper Hessenberg H, by Givens
    rotations and back substitution (plain floats, fixed operation order)."""
    m = H.shape[1]
    R = [[float(H[i, j]) for j in range(m)] for i in range(m + 1)]
    g = [0.0] * (m + 1)
    g[0] = float(beta)
    cs, sn = [], []
    for j in range(m):
        for i in range(j):
            a, b = R[i][j], R[i + 1][j]
            R[i][j] = cs[i] * a + sn[i] * b
            R[i + 1][j] = -sn[i] * a + cs[i] * b
        a, b = R[j][j], R[j + 1][j]
        r = math.sqrt(a * a + b * b)
        if r == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / r, b / r
        cs.append(c)
        sn.append(s)
        R[j][j] = r
        R[j + 1][j] = 0.0
        g[j + 1] = -s * g[j]
        g[j] = c * g[j]
    y = [0.0] * m
    for i in reversed(range(m)):
        t = g[i]
        for k in range(i + 1, m):
            t = t - R[i][k] * y[k]
        y[i] = t / R[i][i]
    return y, abs(g[m])


# ---------------------------------------------------------------------------
# F-point smoother: monomial GMRES polynomial coefficients (Eq. gmres_poly)
# ---------------------------------------------------------------------------

def gmres_poly_coeffs(A, b, degree):
    """alpha_0..alpha_d with q(A) b = sum_i alpha_i A^i b the GMRES iterate after
    d+1 steps from x0 = 0, i.e. the minimiser of |b - A x| over K_{d+1}(A, b).

    The monomial coefficients of every Arnoldi vector are carried along:
    v_1 = b / beta and v_{j+1} = (A v_j - sum_k h_kj v_k) / h_{j+1,j}.
    The degree drops below d on a happy breakdown (an invariant subspace).
    """
    n = A.shape[0]
    m = min(degree + 1, n)
    if m <= 0:
        return np.zeros(0)
    V, H, steps, beta = arnoldi(A, b, m)
    C = np.zeros((steps, steps))
    C[0, 0] = 1.0 / beta
    for j in range(steps - 1):
        c = np.zeros(steps)
        c[1:j + 2] = C[0:j + 1, j]
        for k in range(j + 1):
            c = c - H[k, j] * C[:, k]
        C[:, j + 1] = c / H[j + 1, j]
    y, _ = givens_lstsq(H[:steps + 1, :steps], beta)
    alpha = np.zeros(steps)
    for i in range(steps):
        s = 0.0
        for k in range(steps):
            s = s + y[k] * C[i, k]
        alpha[i] = s
    return alpha


def horner_apply(A, alpha, s):
    """q(A) s = alpha_0 s + alpha_1 A s + ... by Horner: y = alpha_d s, then
    y = A y + alpha_k s for k = d-1 .. 0 (d products with A)."""
    d = len(alpha) - 1
    y = alpha[d] * s
    for k in range(d - 1, -1, -1):
        y = spmv(A, y) + alpha[k] * s
    return y


def neumann_apply(A, d, s):
    """The Jacobi-scaled Neumann polynomial of nAIR (Sec. 3.3's comparison),
    q(A) s = sum_{k=0}^{d} N^k D^{-1} s with D = diag(A), N = I - D^{-1} A,
    applied as y = D^{-1} s, then d times y = y + D^{-1} (s - A y)
    (d products with A)."""
    dinv = 1.0 / A.diagonal()
    y = dinv * s
    for _ in range(d):
        y = y + dinv * (s - spmv(A, y))
    return y


# ---------------------------------------------------------------------------
# Coarse solver: harmonic Ritz roots in Newton form (Sec. 2.3)
# ---------------------------------------------------------------------------

RANK_TOL = 1e-12


def harmonic_ritz(H, k):
    """Harmonic Ritz values of the k-step Arnoldi relation: the eigenvalues of
    H_k + h_{k+1,k}^2 f e_k^T with H_k^T f = e_k.  They are the roots of the
    GMRES residual polynomial."""
    Hk = H[:k, :k]
    h = H[k, k - 1]
    ek = np.zeros(k)
    ek[k - 1] = 1.0
    f = np.linalg.solve(Hk.T, ek)
    M = Hk.copy()
    M[:, k - 1] += h * h * f
    return np.linalg.eigvals(M)


def numerical_rank(Hk):
    """Rank of a square matrix by column-pivoted QR with relative tolerance RANK_TOL."""
    _, R, _ = scipy.linalg.qr(Hk, pivoting=True)
    d = np.abs(np.diag(R))
    if d[0] == 0.0:
        return 0
    return int(np.sum(d > RANK_TOL * d[0]))


def _canon(roots):
    """Real roots get an exactly zero imaginary part; complex roots come as
    exact conjugate pairs.  Returns the list of 'representatives': every real
    root and the Im > 0 member of every pair."""
    reps = [complex(r) for r in roots if r.imag >= 0.0]
    reps.sort(key=lambda z: (z.real, z.imag))
    return reps


def leja_order(roots):
    """Modified Leja ordering: start from the root of largest modulus, then take
    the root that maximises the product of distances to those already taken
    (sums of logs); a complex root is followed at once by its conjugate."""
    reps = _canon(roots)
    taken = []
    out = []
    remaining = list(reps)
    while remaining:
        if not taken:
            scores = [abs(z) for z in remaining]
        else:
            scores = []
            for z in remaining:
                s = 0.0
                for t in taken:
                    d = abs(z - t)
                    s += math.log(d) if d > 0.0 else -math.inf
                scores.append(s)
        best = int(np.argmax(scores))
        z = remaining.pop(best)
        if z.imag == 0.0:
            out.append(z)
            taken.append(z)
        else:
            out.extend([z, z.conjugate()])
            taken.extend([z, z.conjugate()])
    return out


def added_roots(roots):
    """Extra copies of outlying roots for stability (Loe & Morgan 2022): with
    pof(k) = prod_{j != k} |1 - theta_k / theta_j|, a root whose log10 pof
    exceeds 4 gets ceil((log10 pof - 4) / 14) more copies (a complex root adds
    pairs).  Products are taken as sums of log10 to avoid overflow."""
    full = list(roots)
    extra = []
    for z in _canon(roots):
        lp = 0.0
        skipped = False
        for t in full:
            if t == z and not skipped:
                skipped = True
                continue
            d = abs(1.0 - z / t)
            lp += math.log10(d) if d > 0.0 else -math.inf
        if lp > 4.0:
            cnt = int(math.ceil((lp - 4.0) / 14.0))
            for _ in range(cnt):
                if z.imag == 0.0:
                    extra.append(z)
                else:
                    extra.extend([z, z.conjugate()])
    return extra


def newton_roots(A, b, degree, use_added_roots=True):
    """Roots of the degree-`degree` GMRES polynomial on A from right-hand side b,
    Leja ordered (the degree is capped by n - 1 and by a happy breakdown, and cut
    to the numerical rank of H_k)."""
    n = A.shape[0]
    m = min(degree + 1, n)
    _, H, steps, _ = arnoldi(A, b, m)
    k = steps
    r = numerical_rank(H[:k, :k])
    k = max(1, min(k, r))
    theta = harmonic_ritz(H, k)
    roots = list(theta)
    if use_added_roots:
        roots = roots + added_roots(roots)
    return leja_order(roots)


def newton_apply(A, roots, r):
    """x = q(A) r with q(z) = (1 - prod_i (1 - z / theta_i)) / z, applied as in
    Loe & Morgan: x += w / theta, w -= A w / theta for a real root; a conjugate
    pair (a +- ib) is applied in real arithmetic from t = A w.  The last root
    skips the update of w, so m roots cost m - 1 products with A."""
    x = np.zeros_like(r)
    w = r.copy()
    m = len(roots)
    i = 0
    while i < m:
        z = roots[i]
        if z.imag == 0.0:
            a = z.real
            x = x + w / a
            if i < m - 1:
                w = w - spmv(A, w) / a
            i += 1
        else:
            a, b = z.real, z.imag
            mod2 = a * a + b * b
            t = spmv(A, w)
            x = x + (2.0 * a / mod2) * w - t / mod2
            if i + 1 < m - 1:
                u = spmv(A, t)
                w = w - (2.0 * a / mod2) * t + u / mod2
            i += 2
    return x
