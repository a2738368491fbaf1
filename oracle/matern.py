"""Matern (nu = 3/2) prior covariance and its truncated Karhunen-Loeve
expansion by the Nystrom method -- the prior of the paper's elliptic
examples (Sec. 5: a Matern field of smoothness 3/2, unit variance, truncated
to its leading KL terms, which the paper reports as fractions of the prior
variance).

TEST INFRASTRUCTURE ONLY.  Plain numpy in float64; only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP library.

Definitions (the paper names the covariance but not its parameterisation or
a discretisation; these are the readings taken):

* C(r) = sigma2 (1 + sqrt(6) r / lam) exp(-sqrt(6) r / lam): the Matern
  function of smoothness nu = 3/2 whose Bessel argument is 2 sqrt(nu) r / lam.
  With it the leading 3 and 10 terms at lam = 0.65 and the leading 3 and 320
  terms at lam = 0.1 hold the variance fractions the paper prints.
* Nystrom operator: the midpoint rule on an m x m grid of (0,1)^2, m even,
  points P_q = ((a + 1/2)/m, (b + 1/2)/m) with q = b m + a, weights w = 1/m^2;
  the discrete operator is A = w [C(|P_q - P_q'|)].
* Canonical eigenvectors: A commutes with the reflections x1 -> 1 - x1 (Fx)
  and x2 -> 1 - x2 (Fy), so the eigenvectors are taken in the four parity
  classes (sx, sy) of (Fx, Fy), ordered (+,+), (-,+), (+,-), (-,-).  The class
  (+,-) is the class (-,+) with the coordinates swapped, which makes the
  paired eigenvalues exactly equal.  Within a class the eigenvalues are
  simple for the kernels and grids used here.
* Order: lambda descending; exactly equal lambdas by class order.
* Sign: sum_q g_q v_q > 0 with g_q = frac((q + 1)^2 * 0.6180339887498949) - 1/2.
  The quadratic Weyl sequence has no relation under the square's
  reflections (the linear one makes g nearly constant over every reflection
  orbit, so g.v vanishes for modes odd under the diagonal swap).
* Basis: B[k, e] = sqrt(lambda_k) phi_k(c_e), phi_k the Nystrom extension
  phi_k(x) = (1/lambda_k) sum_q w C(|x - P_q|) phi_k(P_q), phi_k(P_q) = v_k[q]/sqrt(w),
  c_e the centroid of element e.
"""
import numpy as np

SQRT6 = np.sqrt(6.0)
GOLDEN_FRAC = 0.6180339887498949
CLASSES = [(1, 1), (-1, 1), (1, -1), (-1, -1)]


def matern32(r, lam, sigma2=1.0):
    """C(r) of the definition above (elementwise over an array of distances)."""
    a = SQRT6 * np.asarray(r, dtype=np.float64) / lam
    return sigma2 * (1.0 + a) * np.exp(-a)


def points(m):
    """Nystrom points, (m*m, 2), q = b m + a."""
    t = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(t, t, indexing="xy")  # X[b, a] = t[a], Y[b, a] = t[b]
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def full_matrix(m, lam, sigma2=1.0):
    """A = w [C(|P_q - P_q'|)], the whole Nystrom operator (M x M)."""
    P = points(m)
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    return matern32(d, lam, sigma2) / (m * m)


def _reps(m):
    """representatives (a, b) with a, b < m/2; block index b (m/2) + a"""
    h = m // 2
    a, b = np.meshgrid(np.arange(h), np.arange(h), indexing="xy")
    return a.ravel(), b.ravel()


def class_matrix(m, lam, sigma2, sx, sy):
    """A restricted to the parity class (sx, sy) in its symmetry-adapted basis:
    A_s[p, p'] = w sum_h chi(h) C(|P_p - P_{h p'}|) over h in {I, Fx, Fy, FxFy}."""
    if m % 2:
        raise ValueError("the Nystrom grid side must be even")
    a, b = _reps(m)
    x, y = (a + 0.5) / m, (b + 0.5) / m
    out = np.zeros((a.size, a.size))
    for fx, cx in ((False, 1), (True, sx)):
        for fy, cy in ((False, 1), (True, sy)):
            xp = 1.0 - x if fx else x
            yp = 1.0 - y if fy else y
            d = np.sqrt((x[:, None] - xp[None, :]) ** 2 + (y[:, None] - yp[None, :]) ** 2)
            out += cx * cy * matern32(d, lam, sigma2)
    return out / (m * m)


def expand(m, v, sx, sy):
    """full-grid vector of a class vector: v_full[g p] = chi(g) v[p] / 2"""
    h = m // 2
    V = v.reshape(h, h)  # [b, a]
    F = np.zeros((m, m))
    F[:h, :h] = V
    F[:h, h:] = sx * V[:, ::-1]          # a -> m-1-a
    F[h:, :h] = sy * V[::-1, :]          # b -> m-1-b
    F[h:, h:] = sx * sy * V[::-1, ::-1]
    return 0.5 * F.ravel()


def _swap(m, v):
    """class vector with the coordinates swapped (a, b) -> (b, a)"""
    h = m // 2
    return v.reshape(h, h).T.ravel()


def modes(K, m, lam, sigma2=1.0):
    """The K leading eigenpairs of the Nystrom operator in the canonical
    basis: (lambda[K], V[M, K] full-grid orthonormal eigenvectors,
    cls[K] class indices)."""
    M = m * m
    if not 1 <= K <= M:
        raise ValueError("need 1 <= K <= m*m")
    cand = []  # (lambda, class index, full vector)
    for c in (0, 1, 3):
        sx, sy = CLASSES[c]
        lam_c, vec_c = np.linalg.eigh(class_matrix(m, lam, sigma2, sx, sy))
        for j in range(lam_c.size):
            cand.append((lam_c[j], c, expand(m, vec_c[:, j], sx, sy)))
            if c == 1:  # the swapped class (+,-): same eigenvalue
                cand.append((lam_c[j], 2, expand(m, _swap(m, vec_c[:, j]), 1, -1)))
    cand.sort(key=lambda t: (-t[0], t[1]))
    q1 = np.arange(M) + 1.0
    g = np.modf(q1 * q1 * GOLDEN_FRAC)[0] - 0.5
    lam_out = np.array([t[0] for t in cand[:K]])
    V = np.zeros((M, K))
    for k, t in enumerate(cand[:K]):
        v = t[2]
        V[:, k] = v if g @ v > 0 else -v
    return lam_out, V, np.array([t[1] for t in cand[:K]])


def centroids(l):
    """element centroids (n_e, 2): element 2(j n + i) is the lower triangle of
    cell (i, j) (vertices (i,j), (i+1,j), (i+1,j+1)), 2(j n + i) + 1 the upper"""
    n = 1 << l
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i, j = i.ravel(), j.ravel()
    c = np.zeros((2 * n * n, 2))
    c[0::2, 0] = (3 * i + 2) / (3 * n)
    c[0::2, 1] = (3 * j + 1) / (3 * n)
    c[1::2, 0] = (3 * i + 1) / (3 * n)
    c[1::2, 1] = (3 * j + 2) / (3 * n)
    return c


def extend(X, lam_k, V, m, lam, sigma2=1.0, chunk=4096):
    """B[k, x] = sqrt(lambda_k) phi_k(x) at the points X (n, 2)."""
    P = points(m)
    w = 1.0 / (m * m)
    out = np.zeros((lam_k.size, X.shape[0]))
    for s in range(0, X.shape[0], chunk):
        Xc = X[s:s + chunk]
        d = np.sqrt(((Xc[:, None, :] - P[None, :, :]) ** 2).sum(-1))
        out[:, s:s + chunk] = (matern32(d, lam, sigma2) @ V).T
    return out * (np.sqrt(w) / np.sqrt(lam_k))[:, None]


def kl_basis(l, K, m, lam, sigma2=1.0):
    """B_l[k, e] = sqrt(lambda_k) phi_k(c_e) for the elements of level l."""
    lam_k, V, _ = modes(K, m, lam, sigma2)
    return extend(centroids(l), lam_k, V, m, lam, sigma2)
