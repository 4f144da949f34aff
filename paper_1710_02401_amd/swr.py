"""Python binding of the SWR C ABI (include/swr.h).

Argument marshalling only: every step of the method runs in libswr.so's HIP
kernels.  PyTorch provides device memory (one caller-owned workspace per
solver) and the HIP stream.  The library must be built in-tree
(paper_1710_02401_amd/libswr.so); loading fails loudly otherwise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswr.so")

(SWR_OK, SWR_E_ARG, SWR_E_SIZE, SWR_E_DEVICE, SWR_E_STATE, SWR_E_SINGULAR, SWR_E_NAN, SWR_E_NOCONV,
 SWR_E_COND) = (0, -1, -2, -3, -4, -5, -6, -7, -8)
SWR_TDSE, SWR_TISE = 0, 1
SWR_WARM_PLAIN, SWR_WARM_ZERO, SWR_WARM_GIVEN = 0, 1, 2
SWR_FACTOR_AUTO, SWR_FACTOR_DIRECT, SWR_FACTOR_WIDE, SWR_FACTOR_BLOCK = 0, 1, 2, 3
SWR_FIELD_SINE, SWR_FIELD_CIRCULAR = 0, 1
SWR_BASIS_GAUSSIAN, SWR_BASIS_SLATER, SWR_BASIS_LSD, SWR_BASIS_LO = 0, 1, 2, 3
MATRICES = {"A": 0, "Kin": 1, "V": 2, "Q": 3, "B": 4, "W": 5, "G": 6, "Q2": 7}

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_f64p = ctypes.POINTER(ctypes.c_double)


class swr_desc(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("n_elec", ctypes.c_int32), ("dim", ctypes.c_int32),
        ("n_geom", ctypes.c_int32), ("L", ctypes.c_int32 * 4),
        ("box_lo", ctypes.c_double * 4), ("box_hi", ctypes.c_double * 4),
        ("overlap", ctypes.c_double * 4),
        ("nbasis", _c_i32p), ("per_subdomain_basis", ctypes.c_int32),
        ("basis_extend", ctypes.c_int32),
        ("width", ctypes.c_double), ("width_ratio", ctypes.c_double),
        ("n_nuc", ctypes.c_int32), ("nuc_pos", _c_f64p), ("nuc_charge", _c_f64p),
        ("eps_en", ctypes.c_double), ("eps_ee", ctypes.c_double),
        ("dt", ctypes.c_double), ("n_steps", ctypes.c_int32),
        ("mu_re", ctypes.c_double), ("mu_im", ctypes.c_double),
        ("E0", ctypes.c_double), ("omega", ctypes.c_double), ("phase", ctypes.c_double),
        ("axis", ctypes.c_int32), ("init_alpha", ctypes.c_double),
        ("init_center", ctypes.c_double * 4),
        ("face_nodes_band", ctypes.c_int32), ("face_nodes_mid", ctypes.c_int32),
        ("quad_nodes", ctypes.c_int32), ("learned_nodes", ctypes.c_int32),
        ("factor_mode", ctypes.c_int32), ("unnormalized", ctypes.c_int32),
        ("field_shape", ctypes.c_int32), ("pulse_nu", ctypes.c_double),
        ("pulse_center", ctypes.c_double), ("field_mask", ctypes.c_int32 * 2),
        ("basis_kind", ctypes.c_int32),
        ("lsd_orbitals", ctypes.c_int32), ("lsd_barrier", ctypes.c_double),
        ("lsd_barrier_width", ctypes.c_double), ("lsd_v_inf", ctypes.c_double),
        ("lsd_moll_eps", ctypes.c_double), ("lsd_moll_order", ctypes.c_int32),
        ("lsd_augment", ctypes.c_int32),
    ]


class swr_info(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32), ("n_sub", ctypes.c_int32), ("n_items", ctypes.c_int32),
        ("K_max", ctypes.c_int32), ("sum_K", ctypes.c_int64), ("sum_K2", ctypes.c_int64),
        ("n_face_nodes", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
        ("sum_KK_pairs", ctypes.c_int64), ("n_steps", ctypes.c_int32),
        ("depth", ctypes.c_int32), ("workspace_bytes", ctypes.c_uint64),
        ("learned_nodes", ctypes.c_int32), ("factor_terms", ctypes.c_int32),
        ("tx_tile", ctypes.c_int32), ("depth_run", ctypes.c_int32), ("wide", ctypes.c_int32),
        ("block", ctypes.c_int32), ("wide_order", ctypes.c_int32), ("tuned", ctypes.c_int32),
        ("rec_series", ctypes.c_int32),
    ]


class swr_run_opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("tol", ctypes.c_double), ("t0", ctypes.c_double),
                ("warm", ctypes.c_int32), ("g_dev", ctypes.c_void_p), ("depth", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("growth_guard", ctypes.c_int32)]


class swr_tuning(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("tx_tile", ctypes.c_int32),
                ("ms_per_window", ctypes.c_double), ("candidates", ctypes.c_int32),
                ("order", ctypes.c_int32)]


class swr_run_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("res", ctypes.c_double * 64), ("energy", ctypes.c_double),
                ("ms_factor", ctypes.c_double), ("ms_transmit", ctypes.c_double),
                ("ms_recur", ctypes.c_double), ("ms_residual", ctypes.c_double),
                ("n_factor", ctypes.c_int32), ("n_transmit", ctypes.c_int32),
                ("n_recur", ctypes.c_int32), ("n_residual", ctypes.c_int32),
                ("fallback", ctypes.c_int32)]


EXPORTS = [
    "swr_create", "swr_destroy", "swr_last_error", "swr_query", "swr_workspace_bytes",
    "swr_bind_workspace", "swr_assemble", "swr_set_initial", "swr_warm_start", "swr_factor",
    "swr_sweep", "swr_transmit", "swr_run", "swr_get_history", "swr_get_forcing",
    "swr_get_initial", "swr_get_matrix", "swr_get_items", "swr_get_terms", "swr_get_boxes",
    "swr_get_index_maps", "swr_get_face_nodes", "swr_reconstruct", "swr_reconstruct_antisym",
    "swr_local_eigen",
    "swr_get_norms", "swr_status_sync", "swr_set_field", "swr_advance_window",
    "swr_time_nodes", "swr_face_data", "swr_learned_features", "swr_learned_targets",
    "swr_learned_apply", "swr_mlp_param_count", "swr_mlp_workspace_bytes", "swr_mlp_forward",
    "swr_mlp_forward_noalloc",
    "swr_mlp_loss_grad", "swr_mlp_adam", "swr_autotune", "swr_set_schedule",
]


class swr_mlp_desc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_layers", ctypes.c_int32), ("n_out", ctypes.c_int32)]

_lib = None


def load_library(path=LIB_PATH):
    """Load libswr.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    vp, i32, u64, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
    sig = {
        "swr_create": (i32, [ctypes.POINTER(swr_desc), ctypes.POINTER(vp)]),
        "swr_destroy": (None, [vp]),
        "swr_last_error": (ctypes.c_char_p, [vp]),
        "swr_query": (i32, [vp, ctypes.POINTER(swr_info)]),
        "swr_workspace_bytes": (i32, [vp, ctypes.POINTER(u64)]),
        "swr_bind_workspace": (i32, [vp, vp, u64]),
        "swr_assemble": (i32, [vp, vp]),
        "swr_set_initial": (i32, [vp, vp, vp]),
        "swr_warm_start": (i32, [vp, i32, vp, vp]),
        "swr_factor": (i32, [vp, ctypes.c_double, vp]),
        "swr_sweep": (i32, [vp, vp]),
        "swr_transmit": (i32, [vp, ctypes.POINTER(ctypes.c_double), vp]),
        "swr_run": (i32, [vp, ctypes.POINTER(swr_run_opts), ctypes.POINTER(swr_run_stats), vp]),
        "swr_autotune": (i32, [vp, i32, ctypes.c_double, ctypes.POINTER(swr_tuning), vp]),
        "swr_set_schedule": (i32, [vp, i32, i32, i32, vp]),
        "swr_get_history": (i32, [vp, vp, u64, vp]),
        "swr_get_forcing": (i32, [vp, vp, u64, vp]),
        "swr_get_initial": (i32, [vp, vp, u64, vp]),
        "swr_get_matrix": (i32, [vp, i32, vp, u64, vp]),
        "swr_get_items": (i32, [vp, _c_i32p, u64]),
        "swr_get_terms": (i32, [vp, _c_i32p, u64]),
        "swr_get_boxes": (i32, [vp, _c_f64p, u64]),
        "swr_get_index_maps": (i32, [vp, _c_i32p, u64]),
        "swr_get_face_nodes": (i32, [vp, _c_f64p, _c_f64p, u64]),
        "swr_reconstruct": (i32, [vp, i32, i32, vp, i64, vp, vp]),
        "swr_reconstruct_antisym": (i32, [vp, i32, i32, vp, i64, vp, vp]),
        "swr_local_eigen": (i32, [vp, vp, vp, vp]),
        "swr_get_norms": (i32, [vp, vp, u64, vp]),
        "swr_status_sync": (i32, [vp, vp]),
        "swr_set_field": (i32, [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
        "swr_advance_window": (i32, [vp, vp]),
        "swr_time_nodes": (i32, [vp, _c_i32p]),
        "swr_face_data": (i32, [vp, i32, _c_i32p, vp, vp]),
        "swr_learned_features": (i32, [vp, vp, ctypes.c_double, i32, vp, vp, vp]),
        "swr_learned_targets": (i32, [vp, vp, vp, i32, vp, vp]),
        "swr_learned_apply": (i32, [vp, vp, vp, vp, i32, vp, vp]),
        "swr_mlp_param_count": (i32, [ctypes.POINTER(swr_mlp_desc), ctypes.POINTER(i64)]),
        "swr_mlp_workspace_bytes": (i32, [ctypes.POINTER(swr_mlp_desc), i32, ctypes.POINTER(u64)]),
        "swr_mlp_forward": (i32, [ctypes.POINTER(swr_mlp_desc), vp, vp, i32, vp, vp, u64, vp]),
        "swr_mlp_forward_noalloc": (i32, [ctypes.POINTER(swr_mlp_desc), vp, vp, i32, vp, vp]),
        "swr_mlp_loss_grad": (i32, [ctypes.POINTER(swr_mlp_desc), vp, vp, vp, i32, vp, vp, vp, u64,
                                    vp]),
        "swr_mlp_adam": (i32, [i64, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SWRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"SWR error {code}: {msg}")
        self.code = code


def _check(lib, h, rc):
    if rc != SWR_OK:
        msg = lib.swr_last_error(h)
        raise SWRError(rc, msg.decode() if msg else "")


def desc_from_config(cfg):
    """swr_desc for a workload dict (see workloads.configs); returns the
    struct and the host arrays it points to (keep them alive)."""
    d = swr_desc()
    D = cfg["n_elec"] * cfg["dim"]
    d.mode = SWR_TISE if cfg["mode"] == "tise" else SWR_TDSE
    d.n_elec, d.dim = cfg["n_elec"], cfg["dim"]
    geoms = cfg.get("geometries")
    d.n_geom = len(geoms) if geoms else 1
    for k in range(D):
        d.L[k] = int(cfg["L"][k])
        d.box_lo[k] = float(cfg["box_lo"][k])
        d.box_hi[k] = float(cfg["box_hi"][k])
        d.overlap[k] = float(cfg["overlap"][k])
    nb = cfg["nbasis"]
    if isinstance(nb[0], (list, tuple)):
        arr = np.ascontiguousarray(np.array(nb, dtype=np.int32).reshape(-1))
        d.per_subdomain_basis = 1
    else:
        arr = np.ascontiguousarray(np.array(nb, dtype=np.int32))
        d.per_subdomain_basis = 0
    d.nbasis = arr.ctypes.data_as(_c_i32p)
    d.basis_extend = int(cfg.get("basis_extend", 0))
    d.width = float(cfg["width"]) if cfg.get("width") is not None else 0.0
    d.width_ratio = float(cfg["width_ratio"]) if cfg.get("width_ratio") is not None else 0.0
    nuclei = geoms if geoms else [cfg["nuclei"]]
    pos = np.ascontiguousarray(np.array(nuclei, dtype=np.float64).reshape(-1))
    chg = np.ascontiguousarray(np.array(cfg["charges"], dtype=np.float64).reshape(-1))
    d.n_nuc = len(cfg["charges"])
    d.nuc_pos = pos.ctypes.data_as(_c_f64p) if pos.size else ctypes.cast(None, _c_f64p)
    d.nuc_charge = chg.ctypes.data_as(_c_f64p) if chg.size else ctypes.cast(None, _c_f64p)
    d.eps_en, d.eps_ee = float(cfg["eps_en"]), float(cfg["eps_ee"])
    d.dt, d.n_steps = float(cfg["dt"]), int(cfg["n_steps"])
    d.mu_re, d.mu_im = float(cfg["mu"][0]), float(cfg["mu"][1])
    f = cfg["field"]
    d.E0, d.omega, d.phase, d.axis = float(f["E0"]), float(f["omega"]), float(f["phase"]), int(f["axis"])
    if f.get("shape", "sine") == "circular":
        # components coupling to the configuration coordinates listed in coords
        d.field_shape = SWR_FIELD_CIRCULAR
        d.pulse_nu, d.pulse_center = float(f["nu"]), float(f["center"])
        for c in range(2):
            d.field_mask[c] = sum(1 << int(k) for k in f["coords"][c])
    elif f.get("shape", "sine") != "sine":
        raise ValueError(f"unknown field shape {f['shape']!r}")
    d.init_alpha = float(cfg["init"]["alpha"])
    for k in range(D):
        d.init_center[k] = float(cfg["init"]["center"][k])
    d.face_nodes_band, d.face_nodes_mid = int(cfg["face_nodes"][0]), int(cfg["face_nodes"][1])
    d.quad_nodes = int(cfg["quad_nodes"])
    d.learned_nodes = int(cfg.get("learned_nodes", 0))
    d.factor_mode = {"auto": SWR_FACTOR_AUTO, "direct": SWR_FACTOR_DIRECT,
                     "wide": SWR_FACTOR_WIDE, "block": SWR_FACTOR_BLOCK}[cfg.get("factor", "auto")]
    d.unnormalized = 1 if cfg.get("unnormalized", False) else 0
    d.basis_kind = {"gaussian": SWR_BASIS_GAUSSIAN, "slater": SWR_BASIS_SLATER,
                    "lsd": SWR_BASIS_LSD, "lo": SWR_BASIS_LO}[cfg.get("basis", "gaussian")]
    pkey = {SWR_BASIS_LSD: "lsd", SWR_BASIS_LO: "lo"}.get(d.basis_kind)
    if pkey in cfg:
        p = cfg[pkey]
        d.lsd_orbitals = int(p["orbitals"])
        d.lsd_barrier = float(p["barrier"])
        d.lsd_barrier_width = float(p["barrier_width"])
        d.lsd_v_inf = float(p["v_inf"])
        d.lsd_moll_eps = float(p["moll_eps"])
        d.lsd_moll_order = int(p["moll_order"])
        d.lsd_augment = int(p.get("augment", 0))
    return d, (arr, pos, chg)


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Solver:
    """One SWR problem on one GPU.  Methods follow the C ABI one to one."""

    def __init__(self, cfg, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.cfg = cfg
        self.device = torch.device(device)
        d, keep = desc_from_config(cfg)
        h = ctypes.c_void_p()
        rc = self.lib.swr_create(ctypes.byref(d), ctypes.byref(h))
        _check(self.lib, None, rc)
        self.h = h
        info = swr_info()
        self._call("swr_query", ctypes.byref(info))
        self.info = info
        self.n_steps = info.n_steps
        items = np.zeros(info.n_items * 10, dtype=np.int32)
        self._call("swr_get_items", items.ctypes.data_as(_c_i32p), ctypes.c_uint64(items.size))
        items = items.reshape(info.n_items, 10)
        self.K = items[:, 0].copy()
        self.n_nodes = items[:, 1].copy()
        self.off1 = np.concatenate([[0], np.cumsum(self.K)]).astype(np.int64)
        self.off2 = np.concatenate([[0], np.cumsum(self.K.astype(np.int64) ** 2)])
        self.stream = stream
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=self.device)
        self._call("swr_bind_workspace", _vp(self.workspace), ctypes.c_uint64(self.workspace.numel()))

    # -- plumbing ------------------------------------------------------------
    def _stream(self):
        if self.stream is not None:
            return ctypes.c_void_p(self.stream.cuda_stream)
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _call(self, name, *args):
        rc = getattr(self.lib, name)(self.h, *args)
        _check(self.lib, self.h, rc)

    def close(self):
        if getattr(self, "h", None):
            self.lib.swr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method ------------------------------------------------------------
    def assemble(self):
        self._call("swr_assemble", self._stream())
        # assembly may take a schedule from the tuning table
        self._call("swr_query", ctypes.byref(self.info))

    def set_initial(self, c0=None):
        self._call("swr_set_initial", _vp(c0), self._stream())

    def warm_start(self, mode=SWR_WARM_PLAIN, g=None):
        self._call("swr_warm_start", ctypes.c_int32(mode), _vp(g), self._stream())

    def factor(self, t0=0.0):
        self._call("swr_factor", ctypes.c_double(t0), self._stream())

    def sweep(self):
        self._call("swr_sweep", self._stream())

    def transmit(self):
        r = ctypes.c_double()
        self._call("swr_transmit", ctypes.byref(r), self._stream())
        return r.value

    def run(self, k_max, tol=0.0, t0=0.0, warm=SWR_WARM_PLAIN, g=None, depth=0, timing=False,
            graph=False, growth_guard=0):
        """swr_run.  Reaching k_max above tol > 0 (SWR_E_NOCONV) is returned as
        converged=False, not raised."""
        o = swr_run_opts(k_max, tol, t0, warm, g.data_ptr() if g is not None else None, depth,
                         int(bool(timing)), int(bool(graph)), int(growth_guard))
        s = swr_run_stats()
        rc = self.lib.swr_run(self.h, ctypes.byref(o), ctypes.byref(s), self._stream())
        if rc != SWR_E_NOCONV:
            _check(self.lib, self.h, rc)
        out = dict(iters=s.iters, converged=bool(s.converged),
                   res=[s.res[i] for i in range(min(s.iters, 64))], energy=s.energy,
                   fallback=bool(s.fallback))
        if timing:
            out["kernels"] = {k: dict(ms=getattr(s, "ms_" + k), launches=getattr(s, "n_" + k))
                              for k in ("factor", "transmit", "recur", "residual")}
        return out

    # -- outputs ---------------------------------------------------------------
    def _complex(self, n):
        return self.torch.empty(int(n), dtype=self.torch.complex128, device=self.device)

    def history(self):
        out = self._complex((self.n_steps + 1) * self.off1[-1])
        self._call("swr_get_history", _vp(out), ctypes.c_uint64(out.numel() * 16), self._stream())
        return out

    def forcing(self):
        out = self._complex((self.n_steps + 1) * self.off1[-1])
        self._call("swr_get_forcing", _vp(out), ctypes.c_uint64(out.numel() * 16), self._stream())
        return out

    def initial(self):
        out = self._complex(self.off1[-1])
        self._call("swr_get_initial", _vp(out), ctypes.c_uint64(out.numel() * 16), self._stream())
        return out

    def split_history(self, flat):
        """List of (n_steps+1, K_s) views, one per item."""
        nT1 = self.n_steps + 1
        return [flat[nT1 * self.off1[s]: nT1 * self.off1[s + 1]].view(nT1, int(self.K[s]))
                for s in range(len(self.K))]

    def split_vector(self, flat):
        return [flat[self.off1[s]: self.off1[s + 1]] for s in range(len(self.K))]

    def matrix(self, which):
        out = self.torch.empty(int(self.off2[-1]), dtype=self.torch.float64, device=self.device)
        self._call("swr_get_matrix", ctypes.c_int32(MATRICES[which]), _vp(out),
                   ctypes.c_uint64(out.numel() * 8), self._stream())
        return [out[self.off2[s]: self.off2[s + 1]].view(int(self.K[s]), int(self.K[s]))
                for s in range(len(self.K))]

    def boxes(self):
        out = np.zeros(len(self.K) * 8)
        self._call("swr_get_boxes", out.ctypes.data_as(_c_f64p), ctypes.c_uint64(out.size))
        return out.reshape(len(self.K), 4, 2)

    def index_maps(self):
        n = int(self.info.n_face_nodes)
        out = np.zeros(n * 16, dtype=np.int32)
        self._call("swr_get_index_maps", out.ctypes.data_as(_c_i32p), ctypes.c_uint64(out.size))
        return out.reshape(n, 16)

    def face_nodes(self):
        n = int(self.info.n_face_nodes)
        x = np.zeros(n * 4)
        w = np.zeros(n)
        self._call("swr_get_face_nodes", x.ctypes.data_as(_c_f64p), w.ctypes.data_as(_c_f64p),
                   ctypes.c_uint64(n))
        return x.reshape(n, 4), w

    def reconstruct(self, pts, step, geom=0, antisym=False):
        pts = pts.to(self.device, dtype=self.torch.float64).contiguous()
        out = self._complex(pts.shape[0])
        fn = "swr_reconstruct_antisym" if antisym else "swr_reconstruct"
        self._call(fn, ctypes.c_int32(geom), ctypes.c_int32(step), _vp(pts),
                   ctypes.c_int64(pts.shape[0]), _vp(out), self._stream())
        return out

    def local_eigen(self):
        lam = self.torch.empty(int(self.off1[-1]), dtype=self.torch.float64, device=self.device)
        X = self.torch.empty(int(self.off2[-1]), dtype=self.torch.float64, device=self.device)
        self._call("swr_local_eigen", _vp(lam), _vp(X), self._stream())
        return ([lam[self.off1[s]: self.off1[s + 1]] for s in range(len(self.K))],
                [X[self.off2[s]: self.off2[s + 1]].view(int(self.K[s]), int(self.K[s]))
                 for s in range(len(self.K))])

    def norms(self):
        out = self.torch.empty(self.n_steps + 1, dtype=self.torch.float64, device=self.device)
        self._call("swr_get_norms", _vp(out), ctypes.c_uint64(out.numel() * 8), self._stream())
        return out

    def status(self):
        self._call("swr_status_sync", self._stream())

    # -- learned warm start plumbing --------------------------------------------
    @property
    def n_face_nodes(self):
        return int(self.info.n_face_nodes)

    def set_field(self, E0, omega, phase):
        self._call("swr_set_field", ctypes.c_double(E0), ctypes.c_double(omega),
                   ctypes.c_double(phase))

    def advance_window(self):
        self._call("swr_advance_window", self._stream())

    def autotune(self, k_iters=3, t0=0.0):
        """Measure every schedule (depth, transmission tile) on this problem and
        keep the fastest for later runs with depth 0."""
        t = swr_tuning()
        self._call("swr_autotune", ctypes.c_int32(k_iters), ctypes.c_double(t0), ctypes.byref(t),
                   self._stream())
        self._call("swr_query", ctypes.byref(self.info))
        return dict(depth=t.depth, tx_tile=t.tx_tile, ms_per_window=t.ms_per_window,
                    candidates=t.candidates, order=t.order)

    def set_schedule(self, depth, tx_tile, order=0):
        """Use this schedule (iterates in flight, transmission tile,
        recurrence order) for later runs with depth 0, without measuring."""
        self._call("swr_set_schedule", ctypes.c_int32(depth), ctypes.c_int32(tx_tile),
                   ctypes.c_int32(order), self._stream())
        self._call("swr_query", ctypes.byref(self.info))

    def factor_terms(self):
        """Series terms - 1 used by the last factorisation (-1: direct inversion)."""
        info = swr_info()
        self._call("swr_query", ctypes.byref(info))
        return int(info.factor_terms)

    def rec_series(self):
        """True when the last factorisation's series is evaluated in each
        recurrence step (no per-step inverses formed)."""
        info = swr_info()
        self._call("swr_query", ctypes.byref(info))
        return bool(info.rec_series)

    def item_terms(self):
        """Series terms each item applies per step after the last factorisation."""
        out = np.zeros(int(self.info.n_items), dtype=np.int32)
        self._call("swr_get_terms", out.ctypes.data_as(_c_i32p), ctypes.c_uint64(out.size))
        return out

    def time_nodes(self):
        out = np.zeros(int(self.info.learned_nodes), dtype=np.int32)
        self._call("swr_time_nodes", out.ctypes.data_as(_c_i32p))
        return [int(v) for v in out]

    def face_data(self, steps):
        steps = np.ascontiguousarray(np.array(steps, dtype=np.int32))
        out = self._complex(len(steps) * self.n_face_nodes)
        self._call("swr_face_data", ctypes.c_int32(len(steps)), steps.ctypes.data_as(_c_i32p),
                   _vp(out), self._stream())
        return out.view(len(steps), self.n_face_nodes)

    def learned_features(self, g0, t0, n_in):
        x = self.torch.empty((len(self.K), n_in), dtype=self.torch.float32, device=self.device)
        sc = self.torch.empty(len(self.K), dtype=self.torch.float64, device=self.device)
        self._call("swr_learned_features", _vp(g0), ctypes.c_double(t0), ctypes.c_int32(n_in),
                   _vp(x), _vp(sc), self._stream())
        return x, sc

    def learned_targets(self, g_nodes, scale, n_out):
        y = self.torch.empty((len(self.K), n_out), dtype=self.torch.float32, device=self.device)
        self._call("swr_learned_targets", _vp(g_nodes), _vp(scale), ctypes.c_int32(n_out), _vp(y),
                   self._stream())
        return y

    def learned_apply(self, y, scale, g0, n_out):
        out = self._complex((self.n_steps + 1) * self.n_face_nodes)
        self._call("swr_learned_apply", _vp(y), _vp(scale), _vp(g0), ctypes.c_int32(n_out),
                   _vp(out), self._stream())
        return out


class Mlp:
    """FP32 network of the learned warm start (kernels in libswr.so)."""

    def __init__(self, n_in, n_hidden, n_layers, n_out, params, device="cuda", max_batch=512):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.d = swr_mlp_desc(n_in, n_hidden, n_layers, n_out)
        cnt = ctypes.c_int64()
        _check(self.lib, None, self.lib.swr_mlp_param_count(ctypes.byref(self.d), ctypes.byref(cnt)))
        self.n_params = cnt.value
        self.device = torch.device(device)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        assert self.params.numel() == self.n_params
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.max_batch = max_batch
        b = ctypes.c_uint64()
        _check(self.lib, None, self.lib.swr_mlp_workspace_bytes(ctypes.byref(self.d),
                                                                 ctypes.c_int32(max_batch),
                                                                 ctypes.byref(b)))
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)

    def _s(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, x):
        x = x.contiguous()
        out = self.torch.empty((x.shape[0], self.d.n_out), dtype=self.torch.float32,
                               device=self.device)
        for a in range(0, x.shape[0], self.max_batch):
            xb = x[a:a + self.max_batch]
            yb = out[a:a + self.max_batch]
            _check(self.lib, None, self.lib.swr_mlp_forward(
                ctypes.byref(self.d), _vp(self.params), _vp(xb), ctypes.c_int32(xb.shape[0]),
                _vp(yb), _vp(self.ws), ctypes.c_uint64(self.ws.numel()), self._s()))
        return out

    def loss_grad(self, x, t):
        assert x.shape[0] <= self.max_batch
        _check(self.lib, None, self.lib.swr_mlp_loss_grad(
            ctypes.byref(self.d), _vp(self.params), _vp(x.contiguous()), _vp(t.contiguous()),
            ctypes.c_int32(x.shape[0]), _vp(self.loss), _vp(self.grad), _vp(self.ws),
            ctypes.c_uint64(self.ws.numel()), self._s()))
        return self.loss, self.grad

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _check(self.lib, None, self.lib.swr_mlp_adam(
            ctypes.c_int64(self.n_params), _vp(self.params), _vp(self.grad), _vp(self.m),
            _vp(self.v), ctypes.c_int32(self.step), ctypes.c_float(lr), ctypes.c_float(b1),
            ctypes.c_float(b2), ctypes.c_float(eps), self._s()))
