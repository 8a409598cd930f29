"""ctypes binding of libhmc (include/hmc.h): argument marshalling only.

Device memory and the stream come from PyTorch; every computation runs in the
library's HIP kernels.  Importing this module does not load the library;
``lib()`` does, and raises if the built ``libhmc.so`` is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmc.so")

HMC_OK = 0
STATUS_EINVAL = -1
STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED", -5: "ENUMERIC"}


class HmcConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box", ctypes.c_double), ("n_sub", ctypes.c_int32),
                ("n_bins", ctypes.c_int32), ("alpha_prior", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("chain_id", ctypes.c_uint32),
                ("n_leapfrog", ctypes.c_int32), ("eps", ctypes.c_double),
                ("fixed_bias_mask", ctypes.c_uint32), ("rj_move", ctypes.c_int32),
                ("rj_log_bound", ctypes.c_double), ("tau_mode", ctypes.c_int32)]


class HmcBuffers(ctypes.Structure):
    _fields_ = [("R", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("delta_k", ctypes.c_void_p),
                ("mom_k", ctypes.c_void_p), ("grad_k", ctypes.c_void_p),
                ("delta_r", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("work_bytes", ctypes.c_size_t), ("growth", ctypes.c_void_p)]


class HmcSweepStats(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("accepted", ctypes.c_int32),
                ("rj_dH", ctypes.c_double), ("rj_accepted", ctypes.c_int32),
                ("rj_wall_hits", ctypes.c_int32),
                ("pk", ctypes.POINTER(ctypes.c_double)),
                ("bias", ctypes.POINTER(ctypes.c_double)),
                ("nbar", ctypes.POINTER(ctypes.c_double))]


EXPORTS = ["hmc_workspace_bytes", "hmc_init", "hmc_init_batch", "leapfrog_trajectory",
           "leapfrog_trajectory_async", "gibbs_sweep_async", "hmc_sweep_record_doubles",
           "hamiltonian", "shell_power", "gibbs_sweep", "hmc_set_state", "hmc_set_params",
           "hmc_set_step", "hmc_warm_start", "hmc_set_launch", "hmc_set_plan", "hmc_get_launch",
           "hmc_autotune", "hmc_set_coefficients", "hmc_get_params", "hmc_shell_index",
           "hmc_set_mass", "hmc_set_mass_diagonal", "hmc_field_moments",
           "hmc_timing", "hmc_use_graph", "hmc_last_error", "hmc_destroy", "shell_power_noalloc",
           "hmc_set_plane_pass",
           "cnn_param_count", "cnn_create", "cnn_get_params", "cnn_forward", "cnn_gradient",
           "cnn_features", "cnn_layer_state",
           "cnn_train_step", "cnn_last_error", "cnn_destroy"]

_lib = None


def lib(path=LIB_PATH):
    """Load libhmc.so (raises FileNotFoundError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with python -m paper_1306_1821_amd.build")
    # PyTorch bundles its own HIP runtime; load it first so that libhmc binds to
    # the same runtime (one HIP runtime per process).
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P, D, I32, U64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_uint64
    L.hmc_workspace_bytes.argtypes = [ctypes.POINTER(HmcConfig)]
    L.hmc_workspace_bytes.restype = ctypes.c_size_t
    L.hmc_init.argtypes = [ctypes.POINTER(HmcConfig), ctypes.POINTER(HmcBuffers), D, D, D, P,
                           ctypes.POINTER(P)]
    L.hmc_init_batch.argtypes = [ctypes.POINTER(HmcConfig), ctypes.POINTER(HmcBuffers), I32, D, D,
                                 D, P, ctypes.POINTER(P)]
    L.leapfrog_trajectory.argtypes = [P, U64, D, ctypes.POINTER(I32)]
    L.hamiltonian.argtypes = [P, I32, D]
    L.leapfrog_trajectory_async.argtypes = [P, U64, P, P]
    L.gibbs_sweep_async.argtypes = [P, U64, P]
    L.hmc_sweep_record_doubles.argtypes = [P]
    L.hmc_sweep_record_doubles.restype = ctypes.c_size_t
    L.shell_power.argtypes = [P, I32, D, ctypes.POINTER(ctypes.c_int64)]
    L.gibbs_sweep.argtypes = [P, U64, ctypes.POINTER(HmcSweepStats)]
    L.hmc_set_state.argtypes = [P, I32, P]
    L.hmc_set_params.argtypes = [P, I32, D, D, D]
    L.hmc_set_step.argtypes = [P, I32, ctypes.c_double]
    L.hmc_warm_start.argtypes = [P, I32, P, P, U64]
    L.hmc_set_launch.argtypes = [P, I32, I32]
    L.hmc_autotune.argtypes = [P, I32, ctypes.POINTER(I32)]
    L.hmc_set_plan.argtypes = [P, I32, I32]
    L.hmc_set_plane_pass.argtypes = [P, I32]
    L.hmc_get_launch.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.hmc_set_coefficients.argtypes = [P, I32, P, P]
    L.hmc_get_params.argtypes = [P, I32, D, D, D]
    L.hmc_shell_index.argtypes = [P, I32, P]
    L.hmc_set_mass.argtypes = [P, I32, P]
    L.hmc_set_mass_diagonal.argtypes = [P, I32, P]
    L.hmc_field_moments.argtypes = [P, I32, P, P, ctypes.c_int64]
    L.hmc_timing.argtypes = [P, I32, D, ctypes.POINTER(ctypes.c_int64)]
    L.hmc_use_graph.argtypes = [P, I32]
    L.hmc_last_error.argtypes = [P]
    L.hmc_last_error.restype = ctypes.c_char_p
    L.hmc_destroy.argtypes = [P]
    L.hmc_destroy.restype = None
    L.shell_power_noalloc.argtypes = [I32, I32, P, P, P, P]
    F = ctypes.POINTER(ctypes.c_float)
    L.cnn_param_count.argtypes = []
    L.cnn_param_count.restype = ctypes.c_size_t
    L.cnn_create.argtypes = [F, P, ctypes.POINTER(P)]
    L.cnn_get_params.argtypes = [P, F]
    L.cnn_forward.argtypes = [P, I32, P, P, P]
    L.cnn_gradient.argtypes = [P, I32, P, P, F, D]
    L.cnn_features.argtypes = [P, I32, P, ctypes.c_float, P, P, P]
    L.cnn_train_step.argtypes = [P, I32, P, P, ctypes.c_float, D]
    L.cnn_layer_state.argtypes = [P, I32, P, P, P]
    L.cnn_last_error.argtypes = [P]
    L.cnn_last_error.restype = ctypes.c_char_p
    L.cnn_destroy.argtypes = [P]
    L.cnn_destroy.restype = None
    for name in EXPORTS:
        if name not in ("hmc_workspace_bytes", "hmc_last_error", "hmc_destroy", "cnn_param_count",
                        "hmc_sweep_record_doubles",
                        "cnn_last_error", "cnn_destroy"):
            getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


class HmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _dptr(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Sampler:
    """One or more chains on one GPU.

    chains: list of dicts with keys n, box, nb, R [c,N,N,N], counts [c,N,N,N]
    (numpy or torch), bias [c], nbar [c], pk [nb] (Mpc/h)^3, and optional
    seed, chain_id, nsteps, eps, alpha_prior, fixed_mask, rj, rj_log_bound,
    tau_mode, delta_k0 (complex [N,N,N/2+1]), growth ([N,N,N] per-voxel growth factor
    of the data model; absent: 1).
    """

    def __init__(self, chains, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.L = lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.chains = []
        cfgs = (HmcConfig * len(chains))()
        bufs = (HmcBuffers * len(chains))()
        bias, nbar, pk = [], [], []
        for i, c in enumerate(chains):
            n, nsub = int(c["n"]), int(np.shape(c["R"])[0])
            cfg = cfgs[i]
            cfg.n, cfg.box, cfg.n_sub, cfg.n_bins = n, float(c["box"]), nsub, int(c["nb"])
            cfg.alpha_prior = float(c.get("alpha_prior", 1.0))
            cfg.seed = int(c.get("seed", 1))
            cfg.chain_id = int(c.get("chain_id", i))
            cfg.n_leapfrog = int(c.get("nsteps", 20))
            cfg.eps = float(c.get("eps", 0.05))
            cfg.fixed_bias_mask = int(c.get("fixed_mask", 1))
            cfg.rj_move = int(bool(c.get("rj", False)))
            cfg.rj_log_bound = float(c.get("rj_log_bound", 10.0))
            cfg.tau_mode = int(bool(c.get("tau_mode", False)))
            wb = self.L.hmc_workspace_bytes(ctypes.byref(cfg))
            if wb == 0:
                raise HmcError(-1, f"invalid configuration for chain {i}")
            f32 = dict(dtype=torch.float32, device=self.device)
            h = n // 2 + 1
            t = dict(
                R=torch.as_tensor(np.asarray(c["R"], dtype=np.float32)).to(self.device).contiguous(),
                counts=torch.as_tensor(np.asarray(c["counts"], dtype=np.float32)).to(self.device).contiguous(),
                delta_k=torch.zeros((n, n, h), dtype=torch.complex64, device=self.device),
                mom_k=torch.zeros((n, n, h), dtype=torch.complex64, device=self.device),
                grad_k=torch.zeros((n, n, h), dtype=torch.complex64, device=self.device),
                delta_r=torch.zeros((n, n, n), **f32),
                alpha=torch.zeros((n, n, n), **f32),
                beta=torch.zeros((n, n, n), **f32),
                work=torch.zeros(wb, dtype=torch.uint8, device=self.device))
            if c.get("growth") is not None:
                t["growth"] = torch.as_tensor(np.asarray(c["growth"], dtype=np.float32)).to(self.device).contiguous()
            if c.get("delta_k0") is not None:
                t["delta_k"].copy_(torch.as_tensor(np.asarray(c["delta_k0"], dtype=np.complex64)))
            b = bufs[i]
            b.R, b.counts = t["R"].data_ptr(), t["counts"].data_ptr()
            b.delta_k, b.mom_k, b.grad_k = (t["delta_k"].data_ptr(), t["mom_k"].data_ptr(),
                                           t["grad_k"].data_ptr())
            b.delta_r, b.alpha, b.beta = t["delta_r"].data_ptr(), t["alpha"].data_ptr(), t["beta"].data_ptr()
            b.work, b.work_bytes = t["work"].data_ptr(), wb
            b.growth = t["growth"].data_ptr() if "growth" in t else None
            bias += list(np.asarray(c["bias"], dtype=np.float64))
            nbar += list(np.asarray(c["nbar"], dtype=np.float64))
            pk += list(np.asarray(c["pk"], dtype=np.float64))
            self.chains.append(dict(n=n, nb=cfg.n_bins, nsub=nsub, box=cfg.box, t=t))
        self._cfgs, self._bufs = cfgs, bufs
        torch.cuda.synchronize(self.device)
        ctx = ctypes.c_void_p()
        st = self.L.hmc_init_batch(cfgs, bufs, len(chains), _dptr(bias), _dptr(nbar), _dptr(pk),
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != HMC_OK:
            raise HmcError(st, self.L.hmc_last_error(None).decode())
        self.ctx = ctx

    # ------------------------------------------------------------------ helpers
    def _check(self, st):
        if st != HMC_OK:
            raise HmcError(st, self.L.hmc_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.L.hmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tensors(self, chain=0):
        return self.chains[chain]["t"]

    # ------------------------------------------------------------------ API
    def trajectory(self, traj_index):
        k = len(self.chains)
        dH = (ctypes.c_double * k)()
        acc = (ctypes.c_int32 * k)()
        self._check(self.L.leapfrog_trajectory(self.ctx, int(traj_index), dH, acc))
        return np.array(dH[:]), np.array(acc[:], dtype=bool)

    def trajectory_async(self, traj_index, dH, accepted):
        """Enqueue a trajectory; dH (float64) and accepted (int32) are device tensors [chains]."""
        self._check(self.L.leapfrog_trajectory_async(self.ctx, int(traj_index),
                                                     ctypes.c_void_p(dH.data_ptr()),
                                                     ctypes.c_void_p(accepted.data_ptr())))

    def sweep_record_size(self):
        return int(self.L.hmc_sweep_record_doubles(self.ctx))

    def sweep_async(self, sweep_index, stats):
        """Enqueue a sweep; stats is a float64 device tensor of sweep_record_size() values."""
        self._check(self.L.gibbs_sweep_async(self.ctx, int(sweep_index),
                                             ctypes.c_void_p(stats.data_ptr())))

    def hamiltonian(self, chain=0):
        out = (ctypes.c_double * 3)()
        self._check(self.L.hamiltonian(self.ctx, chain, out))
        return tuple(out[:])

    def shell_power(self, chain=0):
        nb = self.chains[chain]["nb"]
        sig = (ctypes.c_double * nb)()
        nm = (ctypes.c_int64 * nb)()
        self._check(self.L.shell_power(self.ctx, chain, sig, nm))
        return np.array(sig[:]), np.array(nm[:], dtype=np.int64)

    def sweep(self, sweep_index):
        k = len(self.chains)
        st = (HmcSweepStats * k)()
        self._check(self.L.gibbs_sweep(self.ctx, int(sweep_index), st))
        out = []
        for i, c in enumerate(self.chains):
            s = st[i]
            out.append(dict(dH=s.dH, accepted=bool(s.accepted), rj_dH=s.rj_dH,
                            rj_accepted=bool(s.rj_accepted), rj_wall_hits=int(s.rj_wall_hits),
                            pk=np.array(s.pk[:c["nb"]]), bias=np.array(s.bias[:c["nsub"]]),
                            nbar=np.array(s.nbar[:c["nsub"]])))
        return out

    def set_state(self, chain, delta_r):
        x = delta_r if isinstance(delta_r, self.torch.Tensor) else \
            self.torch.as_tensor(np.asarray(delta_r, dtype=np.float32))
        x = x.to(self.device, dtype=self.torch.float32).contiguous()
        self._check(self.L.hmc_set_state(self.ctx, chain, ctypes.c_void_p(x.data_ptr())))
        self.torch.cuda.synchronize(self.device)

    def field_moments(self, chain, mean, m2, count):
        """Fold the chain's current delta_r into running float64 moments (device
        tensors [N][N][N]); count = number of states including this one."""
        for t in (mean, m2):
            assert t.dtype == self.torch.float64 and t.is_contiguous() and t.device == self.device
        self._check(self.L.hmc_field_moments(self.ctx, int(chain), ctypes.c_void_p(mean.data_ptr()),
                                             ctypes.c_void_p(m2.data_ptr()), int(count)))

    def warm_start(self, chain, mu, logvar, draw_index=0):
        """delta = mu + sqrt(exp(logvar) / sigma^2) x (prior draw x); see hmc_warm_start."""
        f = lambda a: (a if isinstance(a, self.torch.Tensor) else
                       self.torch.as_tensor(np.asarray(a, dtype=np.float32))).to(
            self.device, dtype=self.torch.float32).contiguous()
        m, v = f(mu), f(logvar)
        self._check(self.L.hmc_warm_start(self.ctx, chain, ctypes.c_void_p(m.data_ptr()),
                                          ctypes.c_void_p(v.data_ptr()), int(draw_index)))
        self.torch.cuda.synchronize(self.device)

    def set_params(self, chain, pk=None, bias=None, nbar=None):
        f = lambda a: None if a is None else _dptr(a)
        self._check(self.L.hmc_set_params(self.ctx, chain, f(pk), f(bias), f(nbar)))

    def set_step(self, chain, eps):
        """Leapfrog step size of one chain (all chains if chain is None)."""
        for i in (range(len(self.chains)) if chain is None else [chain]):
            self._check(self.L.hmc_set_step(self.ctx, i, float(eps)))

    def set_coefficients(self, chain, alpha, beta):
        a = self.torch.as_tensor(np.asarray(alpha, dtype=np.float32)).to(self.device).contiguous()
        b = self.torch.as_tensor(np.asarray(beta, dtype=np.float32)).to(self.device).contiguous()
        self._check(self.L.hmc_set_coefficients(self.ctx, chain, ctypes.c_void_p(a.data_ptr()),
                                                ctypes.c_void_p(b.data_ptr())))
        self.torch.cuda.synchronize(self.device)

    def set_mass(self, chain, logvar=None, kind="learned"):
        """Install the learned mass from a log-variance field (None: plain mass);
        chain None: every chain.  kind "diagonal": the real-space diagonal variant
        (inverse mass P diag(exp(logvar)) P, no Fourier preconditioning)."""
        chain = -1 if chain is None else chain
        fn = {"learned": self.L.hmc_set_mass, "diagonal": self.L.hmc_set_mass_diagonal}[kind]
        if logvar is None:
            self._check(fn(self.ctx, chain, None))
            return
        x = logvar if isinstance(logvar, self.torch.Tensor) else \
            self.torch.as_tensor(np.asarray(logvar, dtype=np.float32))
        x = x.to(self.device, dtype=self.torch.float32).contiguous()
        self._check(fn(self.ctx, chain, ctypes.c_void_p(x.data_ptr())))
        self.torch.cuda.synchronize(self.device)

    def get_params(self, chain=0):
        c = self.chains[chain]
        pk = np.zeros(c["nb"])
        b = np.zeros(c["nsub"])
        nb = np.zeros(c["nsub"])
        self._check(self.L.hmc_get_params(self.ctx, chain, _dptr_out(pk), _dptr_out(b), _dptr_out(nb)))
        return pk, b, nb

    def shell_index(self, chain=0):
        n = self.chains[chain]["n"]
        out = self.torch.empty((n, n, n // 2 + 1), dtype=self.torch.int16, device=self.device)
        self._check(self.L.hmc_shell_index(self.ctx, chain, ctypes.c_void_p(out.data_ptr())))
        return out.cpu().numpy()

    def set_launch(self, pass_class, grid):
        """Persistent workgroups for a pass class (0 x, 1 y, 2 z); 0: one per tile;
        -1: one launch per grid size of a mixed-size batch."""
        self._check(self.L.hmc_set_launch(self.ctx, int(pass_class), int(grid)))

    def set_plan(self, pass_class, plan):
        """Radix plan (0, 1, 2) or tile shape (3: twice the threads per pencil at
        64^3, 128^3, 256^3) of a pass class's transforms in single-size launches of
        64^3 .. 256^3 grids; plans other than 0 change rounding."""
        self._check(self.L.hmc_set_plan(self.ctx, int(pass_class), int(plan)))

    def set_plane_pass(self, enable=True):
        """Fused y-z plane pass (grid sizes 64 to 256: single-size contexts and the
        size groups of batches) or separate y, z, y passes."""
        self._check(self.L.hmc_set_plane_pass(self.ctx, int(bool(enable))))

    def launch_config(self):
        """(grids, plans) in force, three of each (pass classes x, y, z)."""
        g, p = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)()
        self._check(self.L.hmc_get_launch(self.ctx, g, p))
        return list(g), list(p)

    def autotune(self, reps=10):
        """Pick the fastest launch grid (then radix plan) per pass class; returns the
        three grids (launch_config() also gives the plans)."""
        out = (ctypes.c_int32 * 3)()
        self._check(self.L.hmc_autotune(self.ctx, int(reps), out))
        return list(out)

    def use_graph(self, enable=True):
        """Replay trajectories / sweeps from captured HIP graphs."""
        self._check(self.L.hmc_use_graph(self.ctx, int(bool(enable))))

    def timing(self, enable=-1):
        """Summed device milliseconds and launch counts of the step passes
        ([0] interior k-space passes, [1] y passes, [2] real-space passes, [3] other).
        enable: 1 all classes, 0x10 | mask | (s << 8) a subset, every (s+1)-th
        launch of a class, 0 stop, -1 read only."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        self._check(self.L.hmc_timing(self.ctx, int(enable), ms, n))
        return np.array(ms[:]), np.array(n[:], dtype=np.int64)

    def state(self, chain=0):
        """Host copies of delta_k, mom_k, grad_k, delta_r, alpha, beta."""
        self.torch.cuda.synchronize(self.device)
        t = self.chains[chain]["t"]
        return {k: t[k].cpu().numpy() for k in ("delta_k", "mom_k", "grad_k", "delta_r", "alpha", "beta")}


def shell_power_noalloc(delta_k, n_bins, sigma, n_modes=None, stream=None):
    """sigma_m (and n_m) of a device half-complex field without a context or any
    allocation (include/hmc.h): delta_k complex64 [N, N, N/2+1], sigma float64
    [n_bins], n_modes int64 [n_bins] or None, all on the current device;
    stream-ordered on `stream` (default: torch's current stream)."""
    import torch
    L = lib()
    n = int(delta_k.shape[0])
    assert delta_k.dtype == torch.complex64 and delta_k.is_contiguous()
    assert sigma.dtype == torch.float64 and sigma.is_contiguous()
    assert n_modes is None or (n_modes.dtype == torch.int64 and n_modes.is_contiguous())
    st = torch.cuda.current_stream(delta_k.device) if stream is None else stream
    r = L.shell_power_noalloc(n, int(n_bins), ctypes.c_void_p(delta_k.data_ptr()),
                              ctypes.c_void_p(sigma.data_ptr()),
                              ctypes.c_void_p(n_modes.data_ptr() if n_modes is not None else None),
                              ctypes.c_void_p(st.cuda_stream))
    if r != HMC_OK:
        raise HmcError(r, L.hmc_last_error(None).decode())


def _dptr_out(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


CNN_LAYERS = [(3, 16), (16, 16), (16, 16), (16, 2)]


def cnn_flatten(params):
    """[(W [27, ci, co], b [co]), ...] -> flat float32 vector (include/cnn.h layout)."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                           np.asarray(b, np.float32).ravel()]) for W, b in params])


def cnn_unflatten(flat):
    out, o = [], 0
    for ci, co in CNN_LAYERS:
        W = flat[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        out.append((W, flat[o:o + co]))
        o += co
    return out


class CNN:
    """The warm-start / mass network (include/cnn.h) on one GPU."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.L = lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        flat = cnn_flatten(params) if isinstance(params, (list, tuple)) else np.asarray(params, np.float32)
        if flat.size != self.L.cnn_param_count():
            raise HmcError(-1, "wrong number of CNN parameters")
        torch.cuda.synchronize(self.device)
        ctx = ctypes.c_void_p()
        st = self.L.cnn_create(flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != HMC_OK:
            raise HmcError(st, self.L.cnn_last_error(None).decode())
        self.ctx = ctx

    def _check(self, st):
        if st != HMC_OK:
            raise HmcError(st, self.L.cnn_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.L.cnn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        return self.torch.as_tensor(np.asarray(a, dtype=np.float32)).to(self.device).contiguous() \
            if not isinstance(a, self.torch.Tensor) else a.contiguous()

    def params(self):
        out = np.zeros(self.L.cnn_param_count(), dtype=np.float32)
        self._check(self.L.cnn_get_params(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def forward(self, inputs):
        """inputs: [3, N, N, N] -> (mu, logvar) device tensors."""
        x = self._dev(inputs)
        n = x.shape[-1]
        mu = self.torch.empty((n, n, n), dtype=self.torch.float32, device=self.device)
        lv = self.torch.empty_like(mu)
        self._check(self.L.cnn_forward(self.ctx, n, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(lv.data_ptr())))
        return mu, lv

    def features(self, beta, beta_scale, mask, sel):
        """[3, N, N, N] device input tensor from beta (device), mask and selection."""
        b, m, s = self._dev(beta), self._dev(mask), self._dev(sel)
        n = b.shape[-1]
        out = self.torch.empty((3, n, n, n), dtype=self.torch.float32, device=self.device)
        self._check(self.L.cnn_features(self.ctx, n, ctypes.c_void_p(b.data_ptr()), float(beta_scale),
                                        ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr())))
        return out

    def gradient(self, inputs, target):
        x, t = self._dev(inputs), self._dev(target)
        g = np.zeros(self.L.cnn_param_count(), dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self.L.cnn_gradient(self.ctx, x.shape[-1], ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(t.data_ptr()),
                                        g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        ctypes.byref(loss)))
        return g, loss.value

    def layer_state(self, layer, n):
        """Host float64 copies (z, a, dz) of layer `layer` from the last gradient
        evaluation on an N^3 grid, each [N^3, C_out] (a is None for layer 3)."""
        cout = CNN_LAYERS[layer][1]
        mk = lambda: self.torch.empty((n ** 3, cout), dtype=self.torch.float32, device=self.device)
        z, dz = mk(), mk()
        a = mk() if layer < 3 else None
        self._check(self.L.cnn_layer_state(self.ctx, int(layer), ctypes.c_void_p(z.data_ptr()),
                                           ctypes.c_void_p(a.data_ptr() if a is not None else None),
                                           ctypes.c_void_p(dz.data_ptr())))
        f = lambda t: None if t is None else t.cpu().numpy().astype(np.float64)
        return f(z), f(a), f(dz)

    def train_step(self, inputs, target, lr):
        x, t = self._dev(inputs), self._dev(target)
        loss = ctypes.c_double()
        self._check(self.L.cnn_train_step(self.ctx, x.shape[-1], ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(t.data_ptr()), float(lr), ctypes.byref(loss)))
        return loss.value
