"""ctypes binding of librjsmc (include/rjsmc.h).  Argument marshalling only.

Every computation runs in the HIP library; torch provides device memory and the
current stream.  If the library is not built, every entry point raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "librjsmc.so")

RJSMC_OK, RJSMC_E_INVALID, RJSMC_E_DEVICE, RJSMC_E_NOMEM, RJSMC_E_CAPACITY, RJSMC_E_UNSUPPORTED = range(6)
RJSMC_F64, RJSMC_F32 = 0, 1
LAYOUT_DECOUPLED, LAYOUT_MERGED = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class RJSMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("rjsmc status %d: %s" % (status, msg))
        self.status = status


class System(ctypes.Structure):
    _fields_ = [("loop_radius_m", ctypes.c_double), ("height_m", ctypes.c_double),
                ("current_a", ctypes.c_double),
                ("n_freq", ctypes.c_int32), ("freq_hz", _dp),
                ("n_hankel", ctypes.c_int32), ("hankel_b", _dp), ("hankel_w", _dp),
                ("n_gate", ctypes.c_int32), ("gate_open_s", _dp), ("gate_close_s", _dp),
                ("eps_mn", ctypes.c_double), ("eps_an", _dp),
                ("kmax_cond", ctypes.c_int32), ("kmax_charg", ctypes.c_int32),
                ("z_max_m", ctypes.c_double), ("fwd_precision", ctypes.c_int32),
                ("max_particles", ctypes.c_int64)]


class Particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("stride", ctypes.c_int64), ("n_per_sounding", ctypes.c_int64),
                ("layout", ctypes.c_int32),
                ("kappa", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
                ("phi_b", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("z_cond", ctypes.c_void_p),
                ("m", ctypes.c_void_p), ("z_charg", ctypes.c_void_p),
                ("log10_tau", ctypes.c_void_p), ("c", ctypes.c_void_p)]


class Prior(ctypes.Structure):
    _fields_ = [("phi_lo", ctypes.c_double), ("phi_hi", ctypes.c_double), ("m_lo", ctypes.c_double),
                ("m_hi", ctypes.c_double), ("ltau_lo", ctypes.c_double), ("ltau_hi", ctypes.c_double),
                ("c_lo", ctypes.c_double), ("c_hi", ctypes.c_double)]


class ReweightArgs(ctypes.Structure):
    _fields_ = [("alpha_tess", ctypes.c_double), ("seed", ctypes.c_uint64), ("step", ctypes.c_int32),
                ("n_sound", ctypes.c_int32), ("step_dev", ctypes.c_void_p)]


N_MOVES = 8


class MutateArgs(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("step", ctypes.c_int32), ("n_moves", ctypes.c_int32),
                ("n_sound", ctypes.c_int32), ("move_prob", ctypes.c_double * N_MOVES),
                ("z_move_sd", ctypes.c_double), ("rw_scale", ctypes.c_double), ("mala_eps", ctypes.c_double),
                ("factors", ctypes.c_void_p), ("prior", Prior), ("step_dev", ctypes.c_void_p),
                ("rw_scale_dev", ctypes.c_void_p), ("stats_sound", ctypes.c_void_p), ("trial", ctypes.c_int32),
                ("zca_birth", ctypes.c_int32), ("mala_eps_dev", ctypes.c_void_p),
                ("keep_gradients", ctypes.c_int32)]


class BisectArgs(ctypes.Structure):
    _fields_ = [("n_sound", ctypes.c_int32), ("init", ctypes.c_int32), ("target", ctypes.c_double),
                ("lo0", ctypes.c_double), ("hi0", ctypes.c_double), ("log_lo", ctypes.c_void_p),
                ("log_hi", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("stats_sound", ctypes.c_void_p)]


class SummaryArgs(ctypes.Structure):
    _fields_ = [("n_sound", ctypes.c_int32), ("n_depth", ctypes.c_int32), ("depth_m", ctypes.c_void_p),
                ("model_count", ctypes.c_void_p), ("log_bfipd", ctypes.c_void_p),
                ("mean_log10_sigma", ctypes.c_void_p), ("mean_m", ctypes.c_void_p), ("p_chargeable", ctypes.c_void_p)]


class PpdArgs(ctypes.Structure):
    _fields_ = [("n_sound", ctypes.c_int32), ("y_obs", ctypes.c_void_p), ("resp", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("sd", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class Archive(ctypes.Structure):
    _fields_ = [("pop", Particles), ("ll", ctypes.c_void_p), ("gamma", ctypes.c_void_p), ("log_z", ctypes.c_void_p),
                ("n_slots", ctypes.c_int32), ("n_used", ctypes.c_int32)]


MAX_ARCHIVE = 64
RJSMC_MAX_PER_SOUNDING = 10240           # particles per sounding of the SMC calls
RJSMC_NOALLOC_MAX_PARTICLES = 262144   # rows of the static scratch of rjsmc_mutate_noalloc


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("layer_sort", ctypes.c_int32),
                ("waves_per_particle", ctypes.c_int32)]


TUNING_CANDIDATES = 16
# (waves_per_block, waves_per_particle); (16, 0) is the spread evaluation
TILE_SHAPES = ((2, 1), (4, 1), (8, 1), (2, 2), (1, 4), (1, 8), (1, 16), (16, 0))


def make_prior(pr):
    return Prior(pr["phi_lo"], pr["phi_hi"], pr["m_lo"], pr["m_hi"], pr["ltau_lo"], pr["ltau_hi"],
                 pr["c_lo"], pr["c_hi"])


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "rjsmc_create": (ctypes.c_int, [ctypes.POINTER(System), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "rjsmc_destroy": (None, [ctypes.c_void_p]),
    "rjsmc_last_error": (ctypes.c_char_p, []),
    "rjsmc_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rjsmc_time_kernel": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "rjsmc_build_time_kernel": (ctypes.c_int, [_dp, ctypes.c_int32, _dp, _dp, ctypes.c_int32, _dp]),
    "rjsmc_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "rjsmc_loglik": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "rjsmc_loglik_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p]),
    "rjsmc_init_prior": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.POINTER(Prior),
                                        ctypes.c_uint64, ctypes.c_void_p]),
    "rjsmc_reweight_resample": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ReweightArgs), ctypes.POINTER(Particles),
                                               ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "rjsmc_adapt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_int32, ctypes.POINTER(Prior),
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "rjsmc_archive_store": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Archive),
                                           ctypes.c_int32, ctypes.c_void_p]),
    "rjsmc_adapt_recycled": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Archive),
                                            ctypes.POINTER(Prior), ctypes.c_void_p, ctypes.c_void_p]),
    "rjsmc_mutate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MutateArgs), ctypes.POINTER(Particles),
                                    ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Particles),
                                    ctypes.POINTER(Particles), ctypes.c_void_p, ctypes.c_void_p]),
    "rjsmc_mutate_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MutateArgs), ctypes.POINTER(Particles),
                                            ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(Particles), ctypes.POINTER(Particles), ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "rjsmc_counter_add": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rjsmc_scale_bisect": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BisectArgs), ctypes.c_void_p]),
    "rjsmc_summarize": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.POINTER(SummaryArgs),
                                       ctypes.c_void_p]),
    "rjsmc_posterior_predictive": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.POINTER(PpdArgs),
                                                  ctypes.c_void_p]),
    "rjsmc_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "rjsmc_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "rjsmc_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Particles), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int32, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_float),
                                      ctypes.c_void_p]),
}


def lib():
    """The loaded librjsmc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librjsmc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != RJSMC_OK:
        raise RJSMCError(status, lib().rjsmc_last_error().decode())


def _as_dp(a):
    return a.ctypes.data_as(_dp)


def build_time_kernel(freq_hz, gate_open_s, gate_close_s):
    """Host-side frequency-to-time matrix of the library, [n_gate, n_freq]."""
    f = np.ascontiguousarray(freq_hz, dtype=np.float64)
    lo = np.ascontiguousarray(gate_open_s, dtype=np.float64)
    hi = np.ascontiguousarray(gate_close_s, dtype=np.float64)
    K = np.zeros((len(lo), len(f)))
    _check(lib().rjsmc_build_time_kernel(_as_dp(f), len(f), _as_dp(lo), _as_dp(hi), len(lo), _as_dp(K)))
    return K


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


_FLOAT_KEYS = ("phi_b", "phi", "z_cond", "m", "z_charg", "log10_tau", "c")


def particles_to_device(p, device="cuda"):
    """Copy a numpy SoA population (see workloads) to device tensors."""
    import torch
    out = {"layout": int(p["layout"]), "n_per_sounding": int(p.get("n_per_sounding", 0))}
    out["kappa"] = torch.as_tensor(np.ascontiguousarray(p["kappa"], dtype=np.int32), device=device)
    out["lambda_"] = torch.as_tensor(np.ascontiguousarray(p["lambda_"], dtype=np.int32), device=device)
    for k in _FLOAT_KEYS:
        out[k] = torch.as_tensor(np.ascontiguousarray(p[k], dtype=np.float64), device=device)
    return out


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def particles_struct(p, n=None, stride=None):
    """Particles struct viewing device tensors of dict p (rows [R, stride])."""
    n_all = int(p["kappa"].shape[0])
    n = n_all if n is None else n
    stride = int(p["phi_b"].shape[-1]) if stride is None else stride
    s = Particles()
    s.n, s.stride, s.n_per_sounding, s.layout = n, stride, int(p.get("n_per_sounding", 0)), int(p["layout"])
    s.kappa, s.lambda_ = _ptr(p["kappa"]), _ptr(p["lambda_"])
    for k in _FLOAT_KEYS:
        setattr(s, k, _ptr(p[k]))
    return s


class Context:
    """A librjsmc context for one acquisition system on one device."""

    def __init__(self, system, device=0, precision="f64", max_particles=0):
        self._ptr = ctypes.c_void_p(0)
        keep = {k: np.ascontiguousarray(system[k], dtype=np.float64)
                for k in ("freq_hz", "hankel_b", "hankel_w", "gate_open_s", "gate_close_s", "eps_an")}
        s = System()
        s.loop_radius_m = system["loop_radius_m"]
        s.height_m = system["height_m"]
        s.current_a = system["current_a"]
        s.n_freq, s.freq_hz = len(keep["freq_hz"]), _as_dp(keep["freq_hz"])
        s.n_hankel, s.hankel_b, s.hankel_w = len(keep["hankel_b"]), _as_dp(keep["hankel_b"]), _as_dp(keep["hankel_w"])
        s.n_gate, s.gate_open_s, s.gate_close_s = len(keep["gate_open_s"]), _as_dp(keep["gate_open_s"]), _as_dp(keep["gate_close_s"])
        s.eps_mn, s.eps_an = system["eps_mn"], _as_dp(keep["eps_an"])
        s.kmax_cond, s.kmax_charg = system["kmax_cond"], system["kmax_charg"]
        s.z_max_m = system["z_max_m"]
        s.fwd_precision = {"f64": RJSMC_F64, "f32": RJSMC_F32}[precision]
        s.max_particles = max_particles
        self.n_gate = s.n_gate
        self.n_freq = s.n_freq
        self.kmax_cond, self.kmax_charg = s.kmax_cond, s.kmax_charg
        self.precision = precision
        self.device = device
        _check(lib().rjsmc_create(ctypes.byref(s), device, ctypes.byref(self._ptr)))

    def close(self):
        if self._ptr:
            lib().rjsmc_destroy(self._ptr)
            self._ptr = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, stream=None):
        _check(lib().rjsmc_check(self._ptr, _stream_handle(stream)))

    def time_kernel(self):
        K = np.zeros((self.n_gate, self.n_freq))
        _check(lib().rjsmc_time_kernel(self._ptr, _as_dp(K)))
        return K

    def summarize(self, p, n_sound, depth_m=None, stream=None):
        """Model counts [S][M], log BFIPD [S] and, on the depth grid (device tensor),
        the model-averaged mean log10 sigma, mean m and P(m > 0) [S][n_depth]."""
        import torch
        dev = p["kappa"].device
        M = (self.kmax_cond + 1) * (self.kmax_charg + 1)
        nd = 0 if depth_m is None else int(depth_m.numel())
        out = {"model_count": torch.empty((n_sound, M), dtype=torch.int32, device=dev),
               "log_bfipd": torch.empty(n_sound, dtype=torch.float64, device=dev),
               "mean_log10_sigma": torch.empty((n_sound, nd), dtype=torch.float64, device=dev),
               "mean_m": torch.empty((n_sound, nd), dtype=torch.float64, device=dev),
               "p_chargeable": torch.empty((n_sound, nd), dtype=torch.float64, device=dev)}
        a = SummaryArgs(n_sound, nd, _ptr(depth_m) if nd else None, _ptr(out["model_count"]), _ptr(out["log_bfipd"]),
                        _ptr(out["mean_log10_sigma"]) if nd else None, _ptr(out["mean_m"]) if nd else None,
                        _ptr(out["p_chargeable"]) if nd else None)
        ps = particles_struct(p)
        _check(lib().rjsmc_summarize(self._ptr, ctypes.byref(ps), ctypes.byref(a), _stream_handle(stream)))
        return out

    def posterior_predictive(self, p, n_sound, y_obs, stream=None):
        """Posterior predictive mean, sd and standardised data [S][n_gate] of each
        sounding's population, and the particles' responses [n][n_gate]."""
        import torch
        dev = p["kappa"].device
        n = int(p["kappa"].shape[0])
        f = lambda *shape: torch.empty(shape, dtype=torch.float64, device=dev)
        out = {"resp": f(n, self.n_gate), "mean": f(n_sound, self.n_gate), "sd": f(n_sound, self.n_gate),
               "z": f(n_sound, self.n_gate)}
        y = y_obs.reshape(n_sound, self.n_gate).contiguous()
        a = PpdArgs(n_sound, _ptr(y), _ptr(out["resp"]), _ptr(out["mean"]), _ptr(out["sd"]), _ptr(out["z"]))
        ps = particles_struct(p)
        _check(lib().rjsmc_posterior_predictive(self._ptr, ctypes.byref(ps), ctypes.byref(a), _stream_handle(stream)))
        return out

    def scale_bisect(self, n_sound, init, target, lo0, hi0, log_lo, log_hi, scale, stats_sound, stream=None):
        a = BisectArgs(n_sound, int(init), target, lo0, hi0, _ptr(log_lo), _ptr(log_hi), _ptr(scale),
                       _ptr(stats_sound))
        _check(lib().rjsmc_scale_bisect(self._ptr, ctypes.byref(a), _stream_handle(stream)))

    def counter_add(self, counter, delta=1, stream=None):
        _check(lib().rjsmc_counter_add(self._ptr, _ptr(counter), int(delta), _stream_handle(stream)))

    # -- tile shape --------------------------------------------------------------------
    def set_tuning(self, waves_per_block, layer_sort, waves_per_particle=1):
        t = Tuning(int(waves_per_block), int(layer_sort), int(waves_per_particle))
        _check(lib().rjsmc_set_tuning(self._ptr, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _check(lib().rjsmc_get_tuning(self._ptr, ctypes.byref(t)))
        return {"waves_per_block": t.waves_per_block, "layer_sort": t.layer_sort,
                "waves_per_particle": t.waves_per_particle}

    def autotune(self, p, y_obs, reps=3, stream=None):
        """Times every tile shape on p, keeps the fastest; returns (best, times_ms)."""
        import torch
        n = int(p["kappa"].shape[0])
        ll = torch.empty(n, dtype=torch.float64, device=p["kappa"].device)
        best = Tuning()
        times = (ctypes.c_float * TUNING_CANDIDATES)()
        ps = particles_struct(p)
        _check(lib().rjsmc_autotune(self._ptr, ctypes.byref(ps), _ptr(y_obs), _ptr(ll), int(reps), ctypes.byref(best),
                                    times, _stream_handle(stream)))
        return ({"waves_per_block": best.waves_per_block, "layer_sort": best.layer_sort,
                 "waves_per_particle": best.waves_per_particle}, list(times))

    # -- hot calls ---------------------------------------------------------------------
    def forward(self, p, out=None, stream=None):
        import torch
        n = int(p["kappa"].shape[0])
        if out is None:
            out = torch.empty((n, self.n_gate), dtype=torch.float64, device=p["kappa"].device)
        ps = particles_struct(p)
        _check(lib().rjsmc_forward(self._ptr, ctypes.byref(ps), _ptr(out), _stream_handle(stream)))
        return out

    def loglik(self, p, y_obs, out=None, stream=None):
        import torch
        n = int(p["kappa"].shape[0])
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=p["kappa"].device)
        ps = particles_struct(p)
        _check(lib().rjsmc_loglik(self._ptr, ctypes.byref(ps), _ptr(y_obs), _ptr(out), _stream_handle(stream)))
        return out

    def loglik_grad(self, p, y_obs, stream=None):
        import torch
        n = int(p["kappa"].shape[0])
        ll = torch.empty(n, dtype=torch.float64, device=p["kappa"].device)
        g = {"layout": p["layout"], "kappa": p["kappa"], "lambda_": p["lambda_"]}
        for k in _FLOAT_KEYS:
            g[k] = torch.zeros_like(p[k])
        ps = particles_struct(p)
        gs = particles_struct(g)
        _check(lib().rjsmc_loglik_grad(self._ptr, ctypes.byref(ps), _ptr(y_obs), _ptr(ll), ctypes.byref(gs),
                                       _stream_handle(stream)))
        return ll, {k: g[k] for k in _FLOAT_KEYS}

    # -- SMC primitives ----------------------------------------------------------------
    def init_prior(self, p, prior, seed, stream=None):
        ps = particles_struct(p)
        pr = make_prior(prior)
        _check(lib().rjsmc_init_prior(self._ptr, ctypes.byref(ps), ctypes.byref(pr), seed, _stream_handle(stream)))

    def reweight_resample(self, p_in, ll_in, p_out, ll_out, gamma, log_z, active, anc, alpha, seed, step, n_sound,
                          stream=None, step_dev=None):
        a = ReweightArgs(alpha, seed, step, n_sound, _ptr(step_dev) if step_dev is not None else None)
        si, so = particles_struct(p_in), particles_struct(p_out)
        _check(lib().rjsmc_reweight_resample(self._ptr, ctypes.byref(a), ctypes.byref(si), _ptr(ll_in),
                                             ctypes.byref(so), _ptr(ll_out), _ptr(gamma), _ptr(log_z), _ptr(active),
                                             _ptr(anc), _stream_handle(stream)))

    def adapt(self, p, n_sound, prior, factors, stream=None):
        ps = particles_struct(p)
        pr = make_prior(prior)
        _check(lib().rjsmc_adapt(self._ptr, ctypes.byref(ps), n_sound, ctypes.byref(pr), _ptr(factors),
                                 _stream_handle(stream)))

    def archive_store(self, p, ll, gamma, log_z, n_sound, archive, slot, stream=None):
        ps = particles_struct(p)
        a = archive.struct()
        _check(lib().rjsmc_archive_store(self._ptr, ctypes.byref(ps), _ptr(ll), _ptr(gamma), _ptr(log_z), n_sound,
                                         ctypes.byref(a), int(slot), _stream_handle(stream)))

    def adapt_recycled(self, p, ll, gamma, log_z, n_sound, archive, prior, factors, stream=None):
        ps = particles_struct(p)
        a = archive.struct()
        pr = make_prior(prior)
        _check(lib().rjsmc_adapt_recycled(self._ptr, ctypes.byref(ps), _ptr(ll), _ptr(gamma), _ptr(log_z), n_sound,
                                          ctypes.byref(a), ctypes.byref(pr), _ptr(factors), _stream_handle(stream)))

    def mutate(self, state, ll, scratch, ll_scratch, gamma, active, y_obs, stats, *, seed, step, n_moves, n_sound,
               prior, move_prob, z_move_sd, rw_scale, factors, mala_eps=0.0, grad_cur=None, grad_prop=None,
               stream=None, step_dev=None, rw_scale_dev=None, stats_sound=None, trial=0, zca_birth=False,
               noalloc=False, mala_eps_dev=None, keep_gradients=False):
        """rjsmc_mutate, or with noalloc=True rjsmc_mutate_noalloc (the library's static
        scratch instead of the context's workspace)."""
        a = MutateArgs()
        a.seed, a.step, a.n_moves, a.n_sound = seed, step, n_moves, n_sound
        for t in range(N_MOVES):
            a.move_prob[t] = float(move_prob[t])
        a.z_move_sd, a.rw_scale, a.mala_eps = z_move_sd, rw_scale, mala_eps
        a.factors = _ptr(factors) if factors is not None else ctypes.c_void_p(0)
        a.prior = make_prior(prior)
        a.step_dev = _ptr(step_dev) if step_dev is not None else None
        a.rw_scale_dev = _ptr(rw_scale_dev) if rw_scale_dev is not None else None
        a.stats_sound = _ptr(stats_sound) if stats_sound is not None else None
        a.trial = int(trial)
        a.zca_birth = 1 if zca_birth else 0
        a.mala_eps_dev = _ptr(mala_eps_dev) if mala_eps_dev is not None else None
        a.keep_gradients = 1 if keep_gradients else 0
        ss, sq = particles_struct(state), particles_struct(scratch)
        gc = ctypes.byref(particles_struct(grad_cur)) if grad_cur is not None else None
        gp = ctypes.byref(particles_struct(grad_prop)) if grad_prop is not None else None
        fn = lib().rjsmc_mutate_noalloc if noalloc else lib().rjsmc_mutate
        _check(fn(self._ptr, ctypes.byref(a), ctypes.byref(ss), _ptr(ll), ctypes.byref(sq), _ptr(ll_scratch),
                  _ptr(gamma), _ptr(active), _ptr(y_obs), gc, gp, _ptr(stats), _stream_handle(stream)))


def empty_device_population(n, kmax_cond, kmax_charg, n_per_sounding=0, device="cuda"):
    """Zeroed DECOUPLED population of device tensors."""
    import torch
    f = lambda *shape: torch.zeros(shape, dtype=torch.float64, device=device)
    return {"layout": LAYOUT_DECOUPLED, "n_per_sounding": n_per_sounding,
            "kappa": torch.zeros(n, dtype=torch.int32, device=device),
            "lambda_": torch.zeros(n, dtype=torch.int32, device=device),
            "phi_b": f(n), "phi": f(kmax_cond, n), "z_cond": f(kmax_cond, n), "m": f(kmax_charg, n),
            "z_charg": f(kmax_charg, n), "log10_tau": f(n), "c": f(n)}


class DeviceArchive:
    """Device buffers of a particle archive of n_slots populations of n particles
    (n_sound soundings); n_used slots are read by Context.adapt_recycled."""

    def __init__(self, n_slots, n, n_sound, kmax_cond, kmax_charg, device="cuda"):
        import torch
        if not 1 <= n_slots <= MAX_ARCHIVE:
            raise ValueError("n_slots must be in 1..%d" % MAX_ARCHIVE)
        M = (kmax_cond + 1) * (kmax_charg + 1)
        self.n_slots, self.n, self.n_sound, self.n_used = n_slots, n, n_sound, 0
        self.pop = empty_device_population(n_slots * n, kmax_cond, kmax_charg, 0, device)
        self.ll = torch.zeros(n_slots * n, dtype=torch.float64, device=device)
        self.gamma = torch.zeros((n_slots, n_sound), dtype=torch.float64, device=device)
        self.log_z = torch.zeros((n_slots, n_sound, M), dtype=torch.float64, device=device)

    def struct(self):
        return Archive(particles_struct(self.pop), _ptr(self.ll), _ptr(self.gamma), _ptr(self.log_z), self.n_slots,
                       self.n_used)


def population_to_host(p):
    out = {"layout": p["layout"], "n_per_sounding": p.get("n_per_sounding", 0)}
    for k, v in p.items():
        if hasattr(v, "cpu"):
            out[k] = v.cpu().numpy()
    return out
