"""ctypes binding of libmls2mc.so.  Argument marshalling only."""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libmls2mc.so")

FP64, MIXED = 0, 1
FIELD_LOG_F64, FIELD_KAPPA_F64, FIELD_KAPPA_F32 = 0, 1, 2
KERNEL_PCN, KERNEL_RWM = 0, 1
SCHEME_MLS2MC, SCHEME_MLB = 0, 1
COV_SEPEXP, COV_MATERN32 = 0, 1
BC_DIRICHLET, BC_FLOW_CELL = 0, 1
DECIDE_ITU, DECIDE_LU, DECIDE_DONE, DECIDE_NEED_CV = 0, 1, 2, 3
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTCONV", 5: "ESINGULAR"}


class Mls2mcError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("l_min", C.c_int), ("l_max", C.c_int), ("K", C.c_int), ("sigma2", C.c_double),
                ("corr_len", C.c_double), ("m", C.c_int), ("sigma_n", C.c_double),
                ("precision", C.c_int), ("rtol", C.c_double), ("max_iters", C.c_int),
                ("cov", C.c_int), ("kl_quad", C.c_int), ("bc", C.c_int)]


class Stage(C.Structure):
    _fields_ = [("l_lo", C.c_int), ("l_hi", C.c_int), ("beta", C.c_double), ("zeta", C.c_double),
                ("s", C.c_double), ("kernel", C.c_int)]


class RunConfig(C.Structure):
    _fields_ = [("J", C.c_int64), ("J_tilde", C.c_int64), ("tau_star", C.c_double),
                ("tau_lu", C.c_double), ("eps", C.c_double), ("n_mcmc", C.c_int),
                ("s_pcn", C.c_double), ("seed", C.c_uint64), ("max_stages", C.c_int),
                ("surrogate", C.c_int), ("sur_collect_max_level", C.c_int),
                ("sur_da_min_level", C.c_int), ("sur_pairs", C.c_int64), ("sur_epochs", C.c_int),
                ("sur_hidden", C.c_int), ("sur_batch", C.c_int), ("sur_lr", C.c_double),
                ("s_adapt", C.c_int), ("scheme", C.c_int), ("tau_min", C.c_double), ("kernel", C.c_int)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class ForwardItem(C.Structure):
    _fields_ = [("l", C.c_int), ("N", C.c_int64), ("theta", C.c_void_p), ("G_out", C.c_void_p),
                ("y", C.c_void_p), ("phi_out", C.c_void_p), ("status_out", C.c_void_p),
                ("iters_out", C.c_void_p)]


class Instance(C.Structure):
    _fields_ = [("J", C.c_int64), ("l_max", C.c_int), ("y", C.c_void_p), ("seed", C.c_uint64),
                ("theta_out", C.c_void_p)]


class RunResult(C.Structure):
    _fields_ = [("n_stages", C.c_int), ("final_level", C.c_int), ("final_beta", C.c_double),
                ("log_Z", C.c_double), ("solves", C.c_int64 * 16), ("accepted", C.c_int64),
                ("proposed", C.c_int64), ("iters_total", C.c_int64), ("not_converged", C.c_int64),
                ("seconds", C.c_double), ("stage1_passed", C.c_int64), ("da_proposed", C.c_int64),
                ("sur_train_seconds", C.c_double), ("sur_final_loss", C.c_double),
                ("graphs_launched", C.c_int64), ("max_stage_log", C.c_int), ("stage_type", _ip),
                ("stage_level", _ip), ("stage_beta", _dp), ("stage_zeta", _dp),
                ("stage_ess", _dp), ("stage_acc_rate", _dp), ("sur_err_mean", C.c_double),
                ("sur_err_max", C.c_double), ("sur_err_count", C.c_int64),
                ("stage_sur_err_mean", _dp), ("stage_sur_err_max", _dp)]


class ProfEntry(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("items", C.c_int64),
                ("iters", C.c_int64)]


PROF_SOLVE, PROF_GEMM = 0, 1
_lib = None
_vp = C.c_void_p


def lib():
    """Load libmls2mc.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing: build the HIP library first "
                              "(python paper_1709_09763_amd/build.py or __graft_entry__.build())")
        L = C.CDLL(library_path)
        L.mls2mc_last_error.restype = C.c_char_p
        L.mls2mc_version.restype = C.c_char_p
        L.mls2mc_n_elem.restype = C.c_int64
        L.mls2mc_n_elem.argtypes = [C.c_int]
        L.mls2mc_n_unknowns.restype = C.c_int64
        L.mls2mc_n_unknowns.argtypes = [C.c_int]
        L.mls2mc_ctx_n_unknowns.restype = C.c_int64
        L.mls2mc_ctx_n_unknowns.argtypes = [_vp, C.c_int]
        L.mls2mc_decide.argtypes = [C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    C.c_double]
        L.mls2mc_n_obs.argtypes = [_vp]
        L.mls2mc_create.argtypes = [C.POINTER(Problem), C.POINTER(_vp)]
        L.mls2mc_destroy.argtypes = [_vp]
        L.mls2mc_kl_field.argtypes = [_vp, C.c_int, C.c_int64, _vp, _vp, C.c_int, _vp]
        L.mls2mc_forward.argtypes = [_vp, C.c_int, C.c_int64, _vp, _vp, _vp, _vp, _vp]
        L.mls2mc_forward_field.argtypes = [_vp, C.c_int, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]
        L.mls2mc_loglik.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp]
        L.mls2mc_next_step.argtypes = [_vp, C.c_int64, _vp, C.c_double, C.c_double, C.c_double,
                                       C.c_double, _vp, _vp, _vp, _vp]
        L.mls2mc_resample.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp]
        L.mls2mc_resample_noalloc.argtypes = [C.c_int64, _vp, _vp, _vp, _vp]
        L.mls2mc_cv_lu.argtypes = [_vp, C.c_int64, _vp, C.c_double, _vp, _vp]
        L.mls2mc_set_linear_model.argtypes = [_vp, _dp, _dp]
        L.mls2mc_set_linear_surrogate.argtypes = [_vp, _dp]
        L.mls2mc_gather.argtypes = [_vp, C.c_int64, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp]
        L.mls2mc_pcn_step.argtypes = [_vp, C.POINTER(Stage), C.c_int64, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp, _vp]
        L.mls2mc_run.argtypes = [_vp, C.POINTER(RunConfig), _vp, _vp, C.POINTER(RunResult), _vp]
        L.mls2mc_philox_fill.argtypes = [_vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_int64, C.c_int, _vp, _vp]
        L.mls2mc_autotune.argtypes = [_vp, C.c_int, C.c_int64, C.POINTER(C.c_double), _vp]
        L.mls2mc_get_launch.argtypes = [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.mls2mc_set_launch.argtypes = [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.mls2mc_surrogate_init.argtypes = [_vp, C.c_int, C.c_int64, C.c_uint64, _vp]
        L.mls2mc_surrogate_n_params.argtypes = [_vp]
        L.mls2mc_surrogate_n_pairs.argtypes = [_vp]
        L.mls2mc_surrogate_n_pairs.restype = C.c_int64
        L.mls2mc_surrogate_set_params.argtypes = [_vp, _vp, _vp]
        L.mls2mc_surrogate_get_params.argtypes = [_vp, _vp, _vp]
        L.mls2mc_surrogate_add_pairs.argtypes = [_vp, C.c_int64, _vp, _vp, _vp]
        L.mls2mc_surrogate_train.argtypes = [_vp, C.c_int, C.c_int, C.c_double, C.c_uint64,
                                             C.POINTER(C.c_float), _vp]
        L.mls2mc_surrogate_predict.argtypes = [_vp, C.c_int64, _vp, _vp, _vp]
        L.mls2mc_surrogate_loss_grad.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp]
        L.mls2mc_pcn_step_da.argtypes = [_vp, C.POINTER(Stage), C.c_int64] + [_vp] * 14
        L.mls2mc_kl_eigenvalues.argtypes = [_vp, C.POINTER(C.c_double)]
        L.mls2mc_forward_batch.argtypes = [_vp, C.c_int, C.POINTER(ForwardItem), _vp]
        L.mls2mc_run_batch.argtypes = [_vp, C.POINTER(RunConfig), C.c_int, C.POINTER(Instance),
                                       C.POINTER(RunResult), C.c_int, _vp]
        L.mls2mc_profile.argtypes = [_vp, C.c_int]
        L.mls2mc_profile_read.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(ProfEntry)]
        _lib = L
    return _lib


def mls2mc_last_error():
    return lib().mls2mc_last_error().decode()


def mls2mc_version():
    return lib().mls2mc_version().decode()


def mls2mc_n_elem(l):
    return lib().mls2mc_n_elem(l)


def mls2mc_n_unknowns(l):
    return lib().mls2mc_n_unknowns(l)


def mls2mc_ctx_n_unknowns(h, l):
    return lib().mls2mc_ctx_n_unknowns(h, l)


def mls2mc_decide(beta, l, l_max, prev_lu, scheme, cv_lu=-1.0, tau_lu=1.0, tau_min=0.0):
    """next update of the update scheme: DECIDE_ITU, DECIDE_LU, DECIDE_DONE or DECIDE_NEED_CV"""
    return lib().mls2mc_decide(float(beta), int(l), int(l_max), int(prev_lu), int(scheme), float(cv_lu),
                               float(tau_lu), float(tau_min))


def _check(rc, where):
    if rc != 0:
        raise Mls2mcError(rc, where, mls2mc_last_error())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor", optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def mls2mc_create(problem: Problem):
    h = C.c_void_p()
    _check(lib().mls2mc_create(C.byref(problem), C.byref(h)), "mls2mc_create")
    return h


def mls2mc_destroy(h):
    _check(lib().mls2mc_destroy(h), "mls2mc_destroy")


def mls2mc_n_obs(h):
    return lib().mls2mc_n_obs(h)


def mls2mc_kl_field(h, l, theta, out, kind):
    N = theta.shape[0]
    dt = torch.float32 if kind == FIELD_KAPPA_F32 else torch.float64
    _check(lib().mls2mc_kl_field(h, l, N, _ptr(theta, torch.float64, name="theta"),
                                 _ptr(out, dt, (N, mls2mc_n_elem(l)), "out"), kind, _stream()),
           "mls2mc_kl_field")


def mls2mc_forward(h, l, theta, G_out, status_out=None, iters_out=None):
    N = theta.shape[0]
    _check(lib().mls2mc_forward(h, l, N, _ptr(theta, torch.float64, name="theta"),
                                _ptr(G_out, torch.float64, (N, mls2mc_n_obs(h)), "G_out"),
                                _ptr(status_out, torch.int8, (N,), "status_out", True),
                                _ptr(iters_out, torch.int32, (N,), "iters_out", True), _stream()),
           "mls2mc_forward")


def mls2mc_forward_field(h, l, kappa, G_out, p_out=None, status_out=None, iters_out=None):
    N = kappa.shape[0]
    _check(lib().mls2mc_forward_field(
        h, l, N, _ptr(kappa, torch.float64, (N, mls2mc_n_elem(l)), "kappa"),
        _ptr(G_out, torch.float64, (N, mls2mc_n_obs(h)), "G_out"),
        _ptr(p_out, torch.float64, (N, mls2mc_ctx_n_unknowns(h, l)), "p_out", True),
        _ptr(status_out, torch.int8, (N,), "status_out", True),
        _ptr(iters_out, torch.int32, (N,), "iters_out", True), _stream()), "mls2mc_forward_field")


def mls2mc_kl_eigenvalues(h, K):
    import numpy as np
    out = np.zeros(K)
    _check(lib().mls2mc_kl_eigenvalues(h, out.ctypes.data_as(_dp)), "mls2mc_kl_eigenvalues")
    return out


def mls2mc_forward_batch(h, items):
    """items: list of dicts l, theta, G_out and optional y, phi_out, status_out, iters_out"""
    arr = (ForwardItem * max(1, len(items)))()
    nobs = mls2mc_n_obs(h)
    for i, it in enumerate(items):
        N = it["theta"].shape[0]
        arr[i].l = it["l"]
        arr[i].N = N
        arr[i].theta = _ptr(it["theta"], torch.float64, name="theta")
        arr[i].G_out = _ptr(it["G_out"], torch.float64, (N, nobs), "G_out")
        arr[i].y = _ptr(it.get("y"), torch.float64, (nobs,), "y", True)
        arr[i].phi_out = _ptr(it.get("phi_out"), torch.float64, (N,), "phi_out", True)
        arr[i].status_out = _ptr(it.get("status_out"), torch.int8, (N,), "status_out", True)
        arr[i].iters_out = _ptr(it.get("iters_out"), torch.int32, (N,), "iters_out", True)
    _check(lib().mls2mc_forward_batch(h, len(items), arr, _stream()), "mls2mc_forward_batch")


def mls2mc_loglik(h, G, y, phi_out):
    N = G.shape[0]
    _check(lib().mls2mc_loglik(h, N, _ptr(G, torch.float64, name="G"),
                               _ptr(y, torch.float64, (mls2mc_n_obs(h),), "y"),
                               _ptr(phi_out, torch.float64, (N,), "phi_out"), _stream()),
           "mls2mc_loglik")


def mls2mc_next_step(h, d, scale, cur, tau_ess, eps, out3, logw_out=None, w_out=None):
    N = d.shape[0]
    _check(lib().mls2mc_next_step(h, N, _ptr(d, torch.float64, (N,), "d"), scale, cur, tau_ess,
                                  eps, _ptr(out3, torch.float64, (3,), "out3"),
                                  _ptr(logw_out, torch.float64, (N,), "logw_out", True),
                                  _ptr(w_out, torch.float64, (N,), "w_out", True), _stream()),
           "mls2mc_next_step")


def mls2mc_cv_lu(h, d, scale, out2):
    N = d.shape[0]
    _check(lib().mls2mc_cv_lu(h, N, _ptr(d, torch.float64, (N,), "d"), scale,
                              _ptr(out2, torch.float64, (2,), "out2"), _stream()), "mls2mc_cv_lu")


def mls2mc_set_linear_surrogate(h, S=None):
    """S: host float64 array of N_obs x K (None: back to the network)"""
    import numpy as np
    if S is None:
        _check(lib().mls2mc_set_linear_surrogate(h, None), "mls2mc_set_linear_surrogate")
        return
    S = np.ascontiguousarray(S, dtype=np.float64)
    if S.ndim != 2 or S.shape[0] != mls2mc_n_obs(h):
        raise ValueError(f"S must be N_obs x K, got {S.shape}")
    _check(lib().mls2mc_set_linear_surrogate(h, S.ctypes.data_as(_dp)), "mls2mc_set_linear_surrogate")


def mls2mc_set_linear_model(h, A=None, E=None):
    """A, E: host float64 arrays of N_obs x K (both or neither)"""
    import numpy as np
    if A is None and E is None:
        _check(lib().mls2mc_set_linear_model(h, None, None), "mls2mc_set_linear_model")
        return
    A = np.ascontiguousarray(A, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    if A.shape != E.shape or A.ndim != 2 or A.shape[0] != mls2mc_n_obs(h):
        raise ValueError(f"A and E must both be N_obs x K, got {A.shape} and {E.shape}")
    _check(lib().mls2mc_set_linear_model(h, A.ctypes.data_as(_dp), E.ctypes.data_as(_dp)),
           "mls2mc_set_linear_model")


def mls2mc_resample(h, w, u, anc_out):
    N = w.shape[0]
    _check(lib().mls2mc_resample(h, N, _ptr(w, torch.float64, (N,), "w"),
                                 _ptr(u, torch.float64, (N,), "u"),
                                 _ptr(anc_out, torch.int32, (N,), "anc_out"), _stream()),
           "mls2mc_resample")


def mls2mc_resample_noalloc(w, u, anc_out):
    """resampling with the library's static scratch (no context, no allocation)"""
    N = w.shape[0]
    _check(lib().mls2mc_resample_noalloc(N, _ptr(w, torch.float64, (N,), "w"),
                                         _ptr(u, torch.float64, (N,), "u"),
                                         _ptr(anc_out, torch.int32, (N,), "anc_out"), _stream()),
           "mls2mc_resample_noalloc")


def mls2mc_gather(h, anc, src, dst):
    N = anc.shape[0]
    ncols = src.shape[1] if src.dim() == 2 else 1
    _check(lib().mls2mc_gather(h, N, ncols, _ptr(anc, torch.int32, (N,), "anc"), src.shape[0],
                               _ptr(src, torch.float64, name="src"),
                               _ptr(dst, torch.float64, name="dst"), _stream()), "mls2mc_gather")


def mls2mc_philox_fill(h, seed, stream_id, stage, sub, out, normal):
    _check(lib().mls2mc_philox_fill(h, seed, stream_id, stage, sub, out.numel(), int(normal),
                                    _ptr(out, torch.float64, name="out"), _stream()),
           "mls2mc_philox_fill")


def mls2mc_pcn_step(h, l_lo, l_hi, beta, zeta, s, theta, G_lo, G_hi, phi_lo, phi_hi, y, xi, u,
                    accepted_out=None, kernel=0):
    N = theta.shape[0]
    st = Stage(l_lo, l_hi, beta, zeta, s, kernel)
    f64 = torch.float64
    _check(lib().mls2mc_pcn_step(
        h, C.byref(st), N, _ptr(theta, f64, name="theta"), _ptr(G_lo, f64, name="G_lo", optional=True),
        _ptr(G_hi, f64, name="G_hi", optional=True), _ptr(phi_lo, f64, name="phi_lo", optional=True),
        _ptr(phi_hi, f64, name="phi_hi", optional=True), _ptr(y, f64, name="y"),
        _ptr(xi, f64, name="xi"), _ptr(u, f64, name="u"),
        _ptr(accepted_out, torch.uint8, (N,), "accepted_out", True), _stream()), "mls2mc_pcn_step")


def _result_dict(res, arrs):
    n = min(res.n_stages, res.max_stage_log)
    out = dict(n_stages=res.n_stages, final_level=res.final_level, final_beta=res.final_beta,
               log_Z=res.log_Z, solves=list(res.solves), accepted=res.accepted,
               proposed=res.proposed, iters_total=res.iters_total,
               not_converged=res.not_converged, seconds=res.seconds,
               stage1_passed=res.stage1_passed, da_proposed=res.da_proposed,
               sur_train_seconds=res.sur_train_seconds, sur_final_loss=res.sur_final_loss,
               graphs_launched=res.graphs_launched, sur_err_mean=res.sur_err_mean,
               sur_err_max=res.sur_err_max, sur_err_count=res.sur_err_count)
    for k, v in arrs.items():
        out[k] = v[:n].copy()
    return out


_STAGE_F64 = ("stage_beta", "stage_zeta", "stage_ess", "stage_acc_rate", "stage_sur_err_mean",
              "stage_sur_err_max")


def _stage_arrays(res, ms):
    import numpy as np
    arrs = dict(stage_type=np.zeros(ms, np.int32), stage_level=np.zeros(ms, np.int32))
    arrs.update({k: np.zeros(ms) for k in _STAGE_F64})
    res.max_stage_log = ms
    res.stage_type = arrs["stage_type"].ctypes.data_as(_ip)
    res.stage_level = arrs["stage_level"].ctypes.data_as(_ip)
    for k in _STAGE_F64:
        setattr(res, k, arrs[k].ctypes.data_as(_dp))
    return arrs


def mls2mc_run_batch(h, cfg: RunConfig, instances, use_graphs=True, max_stage_log=1000):
    """instances: list of dicts J, l_max, y (device), seed, theta_out (device J x K)"""
    n = len(instances)
    inst = (Instance * n)()
    res = (RunResult * n)()
    arrs = []
    for i, d in enumerate(instances):
        inst[i].J = d["J"]
        inst[i].l_max = d["l_max"]
        inst[i].y = _ptr(d["y"], torch.float64, name="y")
        inst[i].seed = d["seed"]
        inst[i].theta_out = _ptr(d["theta_out"], torch.float64, name="theta_out")
        arrs.append(_stage_arrays(res[i], max_stage_log))
    torch.cuda.synchronize()
    _check(lib().mls2mc_run_batch(h, C.byref(cfg), n, inst, res, int(use_graphs), None),
           "mls2mc_run_batch")
    return [_result_dict(res[i], arrs[i]) for i in range(n)]


def mls2mc_run(h, cfg: RunConfig, y, theta_out, max_stage_log=4000):
    res = RunResult()
    arrs = _stage_arrays(res, max_stage_log)
    _check(lib().mls2mc_run(h, C.byref(cfg), _ptr(y, torch.float64, name="y"),
                            _ptr(theta_out, torch.float64, name="theta_out"), C.byref(res),
                            _stream()), "mls2mc_run")
    return _result_dict(res, arrs)


def mls2mc_surrogate_init(h, hidden=256, capacity=20480, seed=0):
    _check(lib().mls2mc_surrogate_init(h, hidden, capacity, seed, _stream()), "mls2mc_surrogate_init")


def mls2mc_surrogate_n_params(h):
    return lib().mls2mc_surrogate_n_params(h)


def mls2mc_surrogate_n_pairs(h):
    return lib().mls2mc_surrogate_n_pairs(h)


def mls2mc_surrogate_set_params(h, params):
    _check(lib().mls2mc_surrogate_set_params(h, _ptr(params, torch.float32, name="params"), _stream()),
           "mls2mc_surrogate_set_params")


def mls2mc_surrogate_get_params(h, params):
    _check(lib().mls2mc_surrogate_get_params(h, _ptr(params, torch.float32, name="params"), _stream()),
           "mls2mc_surrogate_get_params")


def mls2mc_surrogate_add_pairs(h, theta, G):
    _check(lib().mls2mc_surrogate_add_pairs(h, theta.shape[0], _ptr(theta, torch.float64, name="theta"),
                                            _ptr(G, torch.float64, name="G"), _stream()),
           "mls2mc_surrogate_add_pairs")


def mls2mc_surrogate_train(h, epochs, batch=256, lr=1e-3, seed=0):
    losses = (C.c_float * max(1, epochs))()
    _check(lib().mls2mc_surrogate_train(h, epochs, batch, lr, seed, losses, _stream()),
           "mls2mc_surrogate_train")
    return [losses[i] for i in range(epochs)]


def mls2mc_surrogate_predict(h, theta, G_out):
    _check(lib().mls2mc_surrogate_predict(h, theta.shape[0], _ptr(theta, torch.float64, name="theta"),
                                          _ptr(G_out, torch.float64, name="G_out"), _stream()),
           "mls2mc_surrogate_predict")


def mls2mc_surrogate_loss_grad(h, x, t, loss_out, grad_out):
    _check(lib().mls2mc_surrogate_loss_grad(h, x.shape[0], _ptr(x, torch.float64, name="x"),
                                            _ptr(t, torch.float64, name="t"),
                                            _ptr(loss_out, torch.float32, name="loss_out"),
                                            _ptr(grad_out, torch.float32, name="grad_out"), _stream()),
           "mls2mc_surrogate_loss_grad")


def mls2mc_pcn_step_da(h, l_lo, l_hi, beta, zeta, s, theta, G_lo, G_hi, phi_lo, phi_hi, y, xi, u1, u2,
                       accepted_out, stage1_out=None, n_solved_lo=None, n_solved_hi=None):
    st = Stage(l_lo, l_hi, beta, zeta, s, 0)
    f64 = torch.float64
    _check(lib().mls2mc_pcn_step_da(
        h, C.byref(st), theta.shape[0], _ptr(theta, f64, name="theta"),
        _ptr(G_lo, f64, name="G_lo", optional=True), _ptr(G_hi, f64, name="G_hi", optional=True),
        _ptr(phi_lo, f64, name="phi_lo", optional=True), _ptr(phi_hi, f64, name="phi_hi", optional=True),
        _ptr(y, f64, name="y"), _ptr(xi, f64, name="xi"), _ptr(u1, f64, name="u1"), _ptr(u2, f64, name="u2"),
        _ptr(accepted_out, torch.uint8, name="accepted_out"),
        _ptr(stage1_out, torch.uint8, name="stage1_out", optional=True),
        _ptr(n_solved_lo, torch.int64, name="n_solved_lo", optional=True),
        _ptr(n_solved_hi, torch.int64, name="n_solved_hi", optional=True), _stream()), "mls2mc_pcn_step_da")


def mls2mc_autotune(h, l, N):
    ms = C.c_double()
    _check(lib().mls2mc_autotune(h, l, N, C.byref(ms), _stream()), "mls2mc_autotune")
    return ms.value


def mls2mc_get_launch(h, l):
    g, b, nu, lds = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    _check(lib().mls2mc_get_launch(h, l, C.byref(g), C.byref(b), C.byref(nu), C.byref(lds)),
           "mls2mc_get_launch")
    return g.value, b.value, nu.value, lds.value


def mls2mc_set_launch(h, l, grid, block, nu=0, lds_bytes=0):
    _check(lib().mls2mc_set_launch(h, l, grid, block, nu, lds_bytes), "mls2mc_set_launch")


def mls2mc_profile(h, enable):
    _check(lib().mls2mc_profile(h, int(enable)), "mls2mc_profile")


def mls2mc_profile_read(h, kclass, l):
    e = ProfEntry()
    _check(lib().mls2mc_profile_read(h, kclass, l, C.byref(e)), "mls2mc_profile_read")
    return dict(launches=e.launches, ms=e.ms, items=e.items, iters=e.iters)


class Context:
    """Owns one library context; methods mirror the C entry points."""

    def __init__(self, l_min, l_max, K, sigma2=1.0, corr_len=0.3, m=3, sigma_n=0.01,
                 precision=FP64, rtol=0.0, max_iters=0, cov=COV_SEPEXP, kl_quad=0, bc=BC_DIRICHLET):
        self.problem = Problem(l_min, l_max, K, sigma2, corr_len, m, sigma_n, precision, rtol,
                               max_iters, cov, kl_quad, bc)
        self.K = K
        self.h = mls2mc_create(self.problem)
        self.nobs = mls2mc_n_obs(self.h)

    def close(self):
        if self.h is not None:
            mls2mc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def kl_eigenvalues(self):
        return mls2mc_kl_eigenvalues(self.h, self.K)

    def autotune(self, l, N):
        ms = mls2mc_autotune(self.h, l, N)
        return ms, mls2mc_get_launch(self.h, l)

    def get_launch(self, l):
        return mls2mc_get_launch(self.h, l)

    def set_launch(self, l, grid, block, nu=0, lds_bytes=0):
        mls2mc_set_launch(self.h, l, grid, block, nu, lds_bytes)

    def profile(self, enable=True):
        mls2mc_profile(self.h, enable)

    def profile_read(self, kclass, l):
        return mls2mc_profile_read(self.h, kclass, l)

    def kl_field(self, l, theta, kind=FIELD_LOG_F64):
        dt = torch.float32 if kind == FIELD_KAPPA_F32 else torch.float64
        out = torch.empty((theta.shape[0], mls2mc_n_elem(l)), dtype=dt, device=theta.device)
        mls2mc_kl_field(self.h, l, theta, out, kind)
        return out

    def forward(self, l, theta, with_stats=False):
        N = theta.shape[0]
        G = torch.empty((N, self.nobs), dtype=torch.float64, device=theta.device)
        st = torch.empty(N, dtype=torch.int8, device=theta.device)
        it = torch.empty(N, dtype=torch.int32, device=theta.device)
        mls2mc_forward(self.h, l, theta, G, st, it)
        return (G, st, it) if with_stats else G

    def forward_field(self, l, kappa, want_p=False):
        N = kappa.shape[0]
        dev = kappa.device
        G = torch.empty((N, self.nobs), dtype=torch.float64, device=dev)
        p = torch.empty((N, mls2mc_ctx_n_unknowns(self.h, l)), dtype=torch.float64, device=dev) if want_p else None
        st = torch.empty(N, dtype=torch.int8, device=dev)
        it = torch.empty(N, dtype=torch.int32, device=dev)
        mls2mc_forward_field(self.h, l, kappa, G, p, st, it)
        return G, p, st, it

    def loglik(self, G, y):
        phi = torch.empty(G.shape[0], dtype=torch.float64, device=G.device)
        mls2mc_loglik(self.h, G, y, phi)
        return phi

    def next_step(self, d, scale, cur, tau_ess, eps=1e-6):
        N = d.shape[0]
        out3 = torch.empty(3, dtype=torch.float64, device=d.device)
        logw = torch.empty(N, dtype=torch.float64, device=d.device)
        w = torch.empty(N, dtype=torch.float64, device=d.device)
        mls2mc_next_step(self.h, d, scale, cur, tau_ess, eps, out3, logw, w)
        return out3, logw, w

    def cv_lu(self, d, scale):
        """device tensor {ESS, cv^2} of the weights exp(-scale d)"""
        out2 = torch.empty(2, dtype=torch.float64, device=d.device)
        mls2mc_cv_lu(self.h, d, scale, out2)
        return out2

    def set_linear_model(self, A=None, E=None):
        """G_l(theta) = (A + 2^{-2l} E) theta in place of the PDE (None, None: back to the PDE)"""
        if A is not None and A.shape[1] != self.K:
            raise ValueError(f"A must have K = {self.K} columns")
        mls2mc_set_linear_model(self.h, A, E)

    def set_linear_surrogate(self, S=None):
        """the delayed-acceptance first stage uses G~ = S theta (None: back to the network)"""
        if S is not None and S.shape[1] != self.K:
            raise ValueError(f"S must have K = {self.K} columns")
        mls2mc_set_linear_surrogate(self.h, S)

    def resample(self, w, u):
        anc = torch.empty(w.shape[0], dtype=torch.int32, device=w.device)
        mls2mc_resample(self.h, w, u, anc)
        return anc

    def gather(self, anc, src):
        dst = torch.empty((anc.shape[0],) + tuple(src.shape[1:]), dtype=src.dtype, device=src.device)
        mls2mc_gather(self.h, anc, src, dst)
        return dst

    def philox(self, seed, stream_id, stage, sub, n, normal, device="cuda"):
        out = torch.empty(n, dtype=torch.float64, device=device)
        mls2mc_philox_fill(self.h, seed, stream_id, stage, sub, out, normal)
        return out

    def pcn_step(self, l_lo, l_hi, beta, zeta, s, theta, G_lo, G_hi, phi_lo, phi_hi, y, xi, u, kernel=0):
        acc = torch.empty(theta.shape[0], dtype=torch.uint8, device=theta.device)
        mls2mc_pcn_step(self.h, l_lo, l_hi, beta, zeta, s, theta, G_lo, G_hi, phi_lo, phi_hi, y,
                        xi, u, acc, kernel)
        return acc

    def run_batch(self, instances, J_tilde=0, tau_star=1.0, n_mcmc=5, s_pcn=0.5, use_graphs=True):
        cfg = RunConfig(0, J_tilde, tau_star, 0.0, 0.0, n_mcmc, s_pcn, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0.0, 0,
                        0, 0.0, 0)
        for d in instances:
            d.setdefault("theta_out", torch.empty((d["J"], self.K), dtype=torch.float64, device="cuda:0"))
        out = mls2mc_run_batch(self.h, cfg, instances, use_graphs)
        for d, o in zip(instances, out):
            o["theta"] = d["theta_out"]
        return out

    def run(self, y, J, J_tilde=0, tau_star=1.0, tau_lu=0.0, eps=0.0, n_mcmc=5, s_pcn=0.5, seed=0,
            max_stages=0, surrogate=False, sur_collect_max_level=0, sur_da_min_level=0, sur_pairs=0,
            sur_epochs=0, sur_hidden=0, sur_batch=0, sur_lr=0.0, s_adapt=False, scheme=0, tau_min=0.0,
            kernel=0):
        """scheme: SCHEME_MLS2MC or SCHEME_MLB; tau_min > 0: adaptive maximum level;
        kernel: KERNEL_PCN or KERNEL_RWM (s_pcn is then the random-walk step)"""
        cfg = RunConfig(J, J_tilde, tau_star, tau_lu, eps, n_mcmc, s_pcn, seed, max_stages,
                        int(surrogate), sur_collect_max_level, sur_da_min_level, sur_pairs, sur_epochs,
                        sur_hidden, sur_batch, sur_lr, int(s_adapt), int(scheme), float(tau_min), int(kernel))
        theta = torch.empty((J, self.K), dtype=torch.float64, device=y.device)
        out = mls2mc_run(self.h, cfg, y, theta)
        out["theta"] = theta
        return out
