"""ctypes wrapper of the CPU FP64 oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and
its binding) never touches it.  All arrays are float64 numpy arrays,
row-major, particle-major.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i32p = C.POINTER(C.c_int32)


class OracleError(RuntimeError):
    pass


class Config(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("l_min", C.c_int), ("l_max", C.c_int), ("K", C.c_int),
        ("sigma2", C.c_double), ("corr_len", C.c_double), ("m", C.c_int), ("nobs", C.c_int),
        ("sigma_n", C.c_double), ("J", C.c_int64), ("J_tilde", C.c_int64),
        ("tau_ess", C.c_double), ("tau_lu", C.c_double), ("eps", C.c_double),
        ("n_mcmc", C.c_int), ("s_pcn", C.c_double), ("seed", C.c_uint64),
        ("max_stages", C.c_int), ("nthreads", C.c_int),
        ("lin_A", _dp), ("lin_E", _dp), ("da_S", _dp), ("s_adapt", C.c_int), ("scheme", C.c_int),
        ("tau_min", C.c_double), ("kernel", C.c_int),
    ]


class Result(C.Structure):
    _fields_ = [
        ("n_stages", C.c_int), ("log_Z", C.c_double), ("final_level", C.c_int),
        ("final_beta", C.c_double), ("solves", C.c_int64 * 16), ("accepted", C.c_int64),
        ("proposed", C.c_int64), ("stage1_passed", C.c_int64), ("stage_type", _ip), ("stage_level", _ip),
        ("stage_beta", _dp), ("stage_zeta", _dp), ("stage_ess", _dp), ("stage_step", _dp),
        ("stage_acc_rate", _dp), ("max_stage_log", C.c_int),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_normal.restype = C.c_double
        L.orc_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_kl_phi_1d.restype = C.c_double
        L.orc_kl_phi_1d.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_potential.restype = C.c_double
        L.orc_potential.argtypes = [C.c_int, _dp, _dp, C.c_double]
        L.orc_ess.restype = C.c_double
        L.orc_ess.argtypes = [C.c_int64, _dp, C.c_double, C.c_double]
        L.orc_next_step.argtypes = [C.c_int64, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                    _dp, _dp, _dp, _dp, _dp]
        L.orc_mh_accept.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_da_accept.argtypes = [C.c_double] * 6 + [_ip]
        L.orc_forward.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int64,
                                  _dp, _dp, C.c_int]
        L.orc_forward_kappa.argtypes = [C.c_int, C.c_int, C.c_int64, _dp, _dp, _dp, C.c_int]
        L.orc_flow_forward_kappa.argtypes = [C.c_int, C.c_int, C.c_int64, _dp, _dp, _dp, C.c_int]
        L.orc_kl_field.argtypes = [C.c_int, C.c_int, C.c_int64, _dp, _dp, _dp]
        L.orc_resample.argtypes = [C.c_int64, _dp, _dp, _i32p]
        L.orc_pcn_propose.argtypes = [C.c_int64, C.c_int, C.c_double, _dp, _dp, _dp]
        L.orc_rwm_propose.argtypes = [C.c_int64, C.c_int, C.c_double, _dp, _dp, _dp]
        L.orc_run_sampler.argtypes = [C.POINTER(Config), _dp, _dp, C.POINTER(Result)]
        L.orc_mlp_forward.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, C.c_int64, _dp, _dp]
        L.orc_mlp_loss_grad.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, C.c_int64, _dp,
                                        _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


# ---------------------------------------------------------------- random --
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(o)


def uniform(seed, stream, stage, sub, idx):
    return lib().orc_uniform(seed, stream, stage, sub, idx)


def normal(seed, stream, stage, sub, idx):
    return lib().orc_normal(seed, stream, stage, sub, idx)


# -------------------------------------------------------------------- KL --
def kl_roots_1d(nmodes, corr_len):
    om = np.zeros(nmodes)
    mu = np.zeros(nmodes)
    _check(lib().orc_kl_roots_1d(nmodes, C.c_double(corr_len), _d(om), _d(mu)), "kl_roots_1d")
    return om, mu


def kl_phi_1d(omega, corr_len, t):
    return np.array([lib().orc_kl_phi_1d(omega, corr_len, float(x)) for x in np.atleast_1d(t)])


def kl_modes_2d(K, sigma2, corr_len):
    lam = np.zeros(K)
    ix = np.zeros(K, dtype=np.int32)
    iy = np.zeros(K, dtype=np.int32)
    ox = np.zeros(K)
    oy = np.zeros(K)
    _check(lib().orc_kl_modes_2d(K, C.c_double(sigma2), C.c_double(corr_len), _d(lam),
                                 ix.ctypes.data_as(_ip), iy.ctypes.data_as(_ip), _d(ox), _d(oy)),
           "kl_modes_2d")
    return lam, ix, iy, ox, oy


def n_elem(l):
    return 2 * (1 << l) ** 2


def n_unknowns(l):
    return ((1 << l) - 1) ** 2


def kl_basis(l, K, sigma2, corr_len):
    B = np.zeros((K, n_elem(l)))
    _check(lib().orc_kl_basis(l, K, C.c_double(sigma2), C.c_double(corr_len), _d(B)), "kl_basis")
    return B


def kl_field(l, B, theta):
    theta = _f64(theta)
    N, K = theta.shape
    a = np.zeros((N, n_elem(l)))
    _check(lib().orc_kl_field(l, K, N, _d(_f64(B)), _d(theta), _d(a)), "kl_field")
    return a


def centroids(l):
    ne = n_elem(l)
    xy = np.zeros((ne, 2))
    x = C.c_double()
    y = C.c_double()
    for e in range(ne):
        lib().orc_centroid(l, e, C.byref(x), C.byref(y))
        xy[e] = (x.value, y.value)
    return xy


# ------------------------------------------------------------------- FEM --
def assemble_band(l, kappa):
    n = 1 << l
    band = np.zeros((n_unknowns(l), n + 1))
    _check(lib().orc_assemble_band(l, _d(_f64(kappa)), _d(band)), "assemble_band")
    return band


def assemble_dense(l, kappa):
    M = n_unknowns(l)
    A = np.zeros((M, M))
    _check(lib().orc_assemble_dense(l, _d(_f64(kappa)), _d(A)), "assemble_dense")
    return A


def load(l, f_nodal=None):
    b = np.zeros(n_unknowns(l))
    fp = _d(_f64(f_nodal)) if f_nodal is not None else None
    _check(lib().orc_load(l, fp, _d(b)), "load")
    return b


def solve(l, kappa, b):
    p = np.zeros(n_unknowns(l))
    _check(lib().orc_solve(l, _d(_f64(kappa)), _d(_f64(b)), _d(p)), "solve")
    return p


def observe(l, m, p):
    G = np.zeros(m * m)
    _check(lib().orc_observe(l, m, _d(_f64(p)), _d(G)), "observe")
    return G


def potential(G, y, sigma_n):
    G = _f64(G)
    y = _f64(y)
    return lib().orc_potential(len(y), _d(G), _d(y), sigma_n)


def forward(l, K, sigma2, corr_len, m, theta, nthreads=0):
    theta = _f64(theta)
    N = theta.shape[0]
    G = np.zeros((N, m * m))
    _check(lib().orc_forward(l, K, sigma2, corr_len, m, N, _d(theta), _d(G), nthreads), "forward")
    return G


def forward_kappa(l, m, kappa, want_p=False, nthreads=0):
    kappa = _f64(kappa)
    N = kappa.shape[0]
    G = np.zeros((N, m * m))
    p = np.zeros((N, n_unknowns(l))) if want_p else None
    _check(lib().orc_forward_kappa(l, m, N, _d(kappa), _d(G), _d(p) if want_p else None, nthreads),
           "forward_kappa")
    return (G, p) if want_p else G


def flow_forward_kappa(l, m, kappa, want_p=False, nthreads=0):
    """flow cell (Example 5.3) by banded Cholesky: G and optionally the
    unknowns' pressure, u = j (n-1) + (i-1) for 1 <= i <= n-1, 0 <= j <= n"""
    kappa = _f64(np.atleast_2d(kappa))
    N = kappa.shape[0]
    n = 1 << l
    G = np.zeros((N, m * m))
    p = np.zeros((N, (n - 1) * (n + 1))) if want_p else None
    _check(lib().orc_flow_forward_kappa(l, m, N, _d(kappa), _d(G), _d(p) if want_p else None, nthreads),
           "flow_forward_kappa")
    return (G, p) if want_p else G


# ------------------------------------------------------------------- SMC --
def ess(d, scale, t):
    d = _f64(d)
    return lib().orc_ess(len(d), _d(d), scale, t)


def next_step(d, scale, cur, tau_ess, eps=1e-6):
    d = _f64(d)
    N = len(d)
    nxt = C.c_double()
    dlz = C.c_double()
    e = C.c_double()
    lw = np.zeros(N)
    w = np.zeros(N)
    _check(lib().orc_next_step(N, _d(d), scale, cur, tau_ess, eps, C.byref(nxt), _d(lw), _d(w),
                               C.byref(dlz), C.byref(e)), "next_step")
    return dict(next=nxt.value, logw=lw, w=w, dlogZ=dlz.value, ess=e.value)


def resample(w, u):
    w = _f64(w)
    u = _f64(u)
    anc = np.zeros(len(u), dtype=np.int32)
    if len(w) != len(u):
        raise OracleError("resample expects len(w) == len(u)")
    _check(lib().orc_resample(len(w), _d(w), _d(u), anc.ctypes.data_as(_i32p)), "resample")
    return anc


def pcn_propose(theta, xi, s):
    theta = _f64(theta)
    out = np.zeros_like(theta)
    N, K = theta.shape
    lib().orc_pcn_propose(N, K, s, _d(theta), _d(_f64(xi)), _d(out))
    return out


def rwm_propose(s, theta, xi):
    theta = _f64(theta)
    out = np.zeros_like(theta)
    N, K = theta.shape
    lib().orc_rwm_propose(N, K, s, _d(theta), _d(_f64(xi)), _d(out))
    return out


def mh_accept(psi_old, psi_new, u):
    return bool(lib().orc_mh_accept(psi_old, psi_new, u))


def da_accept(psi_old, psi_new, psis_old, psis_new, u1, u2):
    s1 = C.c_int()
    a = lib().orc_da_accept(psi_old, psi_new, psis_old, psis_new, u1, u2, C.byref(s1))
    return bool(a), bool(s1.value)


def run_sampler(y, *, model="pde", l_min=4, l_max=4, K=10, sigma2=1.0, corr_len=0.3, m=3,
                nobs=None, sigma_n=0.01, J=200, J_tilde=None, tau_star=1.0, tau_lu=None,
                eps=1e-6, n_mcmc=5, s_pcn=0.5, seed=0, max_stages=2000, nthreads=0,
                lin_A=None, lin_E=None, da_S=None, s_adapt=False, scheme=0, tau_min=0.0, kernel=0):
    """Run the MLS^2MC sampler; returns a dict of results and final particles."""
    y = _f64(y)
    cfg = Config()
    cfg.model = {"pde": 0, "linear": 1, "flowcell": 2}[model]
    cfg.l_min, cfg.l_max, cfg.K = l_min, l_max, K
    cfg.sigma2, cfg.corr_len, cfg.m = sigma2, corr_len, m
    cfg.nobs = nobs if nobs is not None else len(y)
    cfg.sigma_n = sigma_n
    cfg.J = J
    cfg.J_tilde = J_tilde if J_tilde is not None else min(100, J)
    cfg.tau_ess = J / (1.0 + tau_star ** 2)
    cfg.tau_lu = tau_lu if tau_lu is not None else tau_star
    cfg.eps, cfg.n_mcmc, cfg.s_pcn, cfg.seed = eps, n_mcmc, s_pcn, seed
    cfg.max_stages, cfg.nthreads = max_stages, nthreads
    cfg.s_adapt = int(s_adapt)
    cfg.scheme, cfg.tau_min, cfg.kernel = int(scheme), float(tau_min), int(kernel)
    keep = []
    if lin_A is not None:
        A = _f64(lin_A)
        E = _f64(lin_E)
        keep += [A, E]
        cfg.lin_A = _d(A)
        cfg.lin_E = _d(E)
    if da_S is not None:
        S = _f64(da_S)
        keep.append(S)
        cfg.da_S = _d(S)
    res = Result()
    ms = max_stages
    st = np.zeros(ms, dtype=np.int32)
    sl = np.zeros(ms, dtype=np.int32)
    sb = np.zeros(ms)
    sz = np.zeros(ms)
    se = np.zeros(ms)
    ss = np.zeros(ms)
    sa = np.zeros(ms)
    res.stage_step = _d(ss)
    res.stage_acc_rate = _d(sa)
    res.stage_type = st.ctypes.data_as(_ip)
    res.stage_level = sl.ctypes.data_as(_ip)
    res.stage_beta = _d(sb)
    res.stage_zeta = _d(sz)
    res.stage_ess = _d(se)
    res.max_stage_log = ms
    theta = np.zeros((J, K))
    _check(lib().orc_run_sampler(C.byref(cfg), _d(y), _d(theta), C.byref(res)), "run_sampler")
    n = min(res.n_stages, ms)
    return dict(theta=theta, log_Z=res.log_Z, n_stages=res.n_stages, final_level=res.final_level,
                final_beta=res.final_beta, solves=list(res.solves), accepted=res.accepted,
                proposed=res.proposed, stage1_passed=res.stage1_passed, stage_type=st[:n].copy(), stage_level=sl[:n].copy(),
                stage_beta=sb[:n].copy(), stage_zeta=sz[:n].copy(), stage_ess=se[:n].copy(),
                stage_step=ss[:n].copy(), stage_acc_rate=sa[:n].copy())


# ------------------------------------------------------------------- MLP --
def mlp_forward(dims, params, x):
    D, H1, H2, O = dims
    x = _f64(x)
    out = np.zeros((x.shape[0], O))
    _check(lib().orc_mlp_forward(D, H1, H2, O, _d(_f64(params)), x.shape[0], _d(x), _d(out)),
           "mlp_forward")
    return out


def mlp_loss_grad(dims, params, x, target):
    D, H1, H2, O = dims
    x = _f64(x)
    params = _f64(params)
    g = np.zeros_like(params)
    loss = C.c_double()
    _check(lib().orc_mlp_loss_grad(D, H1, H2, O, _d(params), x.shape[0], _d(x),
                                   _d(_f64(target)), C.byref(loss), _d(g)), "mlp_loss_grad")
    return loss.value, g
