"""Flow-cell forward problem (Sec. 5, Example 5.3): P1 finite elements for

    -div(kappa grad p) = 0  on (0,1)^2,
    p = 0 on x1 = 0,   p = 1 on x1 = 1,   dp/dn = 0 on x2 = 0 and x2 = 1,

on the uniform mesh of level l (n = 2^l cells per side, each cut from (i,j)
to (i+1,j+1); element 2(j n + i) is the lower triangle, 2(j n + i) + 1 the
upper), kappa constant per element, and the pressure observed at the points
(a/(m+1), b/(m+1)) by P1 interpolation.

TEST INFRASTRUCTURE ONLY.  Plain numpy / scipy in float64; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the HIP library.

The stiffness matrix is assembled triangle by triangle from the gradients
of the barycentric coordinates (no use of the mesh's right angles); the
Dirichlet nodes are eliminated and the system is solved by a sparse direct
solver.  Unknowns: nodes (i, j) with 1 <= i <= n-1, 0 <= j <= n, index
u = j (n - 1) + (i - 1).
"""
import numpy as np
from scipy import sparse
from scipy.sparse import linalg as splinalg


def n_unknowns(l):
    n = 1 << l
    return (n - 1) * (n + 1)


def elements(l):
    """vertex node indices (n_e, 3), node index j (n+1) + i"""
    n = 1 << l
    s = n + 1
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i, j = i.ravel(), j.ravel()
    a = j * s + i
    tri = np.zeros((2 * n * n, 3), dtype=np.int64)
    tri[0::2] = np.stack([a, a + 1, a + s + 1], 1)   # lower: (i,j), (i+1,j), (i+1,j+1)
    tri[1::2] = np.stack([a, a + s, a + s + 1], 1)   # upper: (i,j), (i,j+1), (i+1,j+1)
    return tri


def node_xy(l):
    n = 1 << l
    t = np.arange(n + 1) / n
    X, Y = np.meshgrid(t, t, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], 1)


def assemble(l, kappa):
    """stiffness matrix over all (n+1)^2 nodes (natural boundary conditions)"""
    xy = node_xy(l)
    tri = elements(l)
    P = xy[tri]  # (n_e, 3, 2)
    x, y = P[..., 0], P[..., 1]
    area2 = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    # grad lambda_a = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1}) / area2
    gx = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], 1) / area2[:, None]
    gy = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], 1) / area2[:, None]
    area = 0.5 * np.abs(area2)
    Kl = (gx[:, :, None] * gx[:, None, :] + gy[:, :, None] * gy[:, None, :]) * (np.asarray(kappa) * area)[:, None, None]
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    N = xy.shape[0]
    return sparse.coo_matrix((Kl.ravel(), (rows, cols)), shape=(N, N)).tocsr()


def solve_nodes(l, kappa):
    """nodal pressure (n+1)^2 of one coefficient field"""
    n = 1 << l
    A = assemble(l, kappa)
    xy = node_xy(l)
    i = np.rint(xy[:, 0] * n).astype(int)
    dirichlet = (i == 0) | (i == n)
    g = np.where(i == n, 1.0, 0.0)
    free = ~dirichlet
    rhs = -(A[free][:, dirichlet] @ g[dirichlet])
    p = g.copy()
    p[free] = splinalg.spsolve(A[free][:, free].tocsc(), rhs)
    return p


def unknowns_of(l, p_nodes):
    """the unknown nodes' values in the order u = j (n-1) + (i-1)"""
    n = 1 << l
    return p_nodes.reshape(n + 1, n + 1)[:, 1:n].ravel()


def observation_weights(l, m):
    """(m*m, 3) node indices and P1 weights of the points (a/(m+1), b/(m+1)),
    o = (b-1) m + (a-1); a point on a diagonal goes to the lower triangle"""
    n = 1 << l
    s = n + 1
    idx = np.zeros((m * m, 3), dtype=np.int64)
    w = np.zeros((m * m, 3))
    for b in range(1, m + 1):
        for a in range(1, m + 1):
            o = (b - 1) * m + (a - 1)
            X, Y = a / (m + 1) * n, b / (m + 1) * n
            i, j = min(int(np.floor(X)), n - 1), min(int(np.floor(Y)), n - 1)
            xi, eta = X - i, Y - j
            c = j * s + i
            if xi >= eta:  # lower: (i,j), (i+1,j), (i+1,j+1)
                idx[o] = (c, c + 1, c + s + 1)
                w[o] = (1.0 - xi, xi - eta, eta)
            else:          # upper: (i,j), (i,j+1), (i+1,j+1)
                idx[o] = (c, c + s, c + s + 1)
                w[o] = (1.0 - eta, eta - xi, xi)
    return idx, w


def forward_kappa(l, m, kappa, want_p=False):
    """G (N, m*m) and, if asked, the unknowns' pressure (N, (n-1)(n+1))"""
    kappa = np.atleast_2d(np.asarray(kappa, dtype=np.float64))
    idx, w = observation_weights(l, m)
    G = np.zeros((kappa.shape[0], m * m))
    P = np.zeros((kappa.shape[0], n_unknowns(l))) if want_p else None
    for q in range(kappa.shape[0]):
        p = solve_nodes(l, kappa[q])
        G[q] = (p[idx] * w).sum(1)
        if want_p:
            P[q] = unknowns_of(l, p)
    return (G, P) if want_p else G
