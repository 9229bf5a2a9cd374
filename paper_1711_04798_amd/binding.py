"""Thin ctypes binding of libctm.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; torch only
supplies device memory (the workspace and the tensor copies) and the stream.
The binding raises if the shared library is missing: there is no CPU path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctm.so")
# launch-variant table written by tune.py on an MI355X (loaded with the library)
TILE_TABLE = os.path.join(_HERE, "tiles.json")

CTM_OK, CTM_E_INVALID, CTM_E_NONFINITE, CTM_E_NOMEM, CTM_E_NOCONV, CTM_E_SOLVER, CTM_E_HIP, CTM_E_STATE = range(8)
STATUS_NAMES = ["OK", "INVALID", "NONFINITE", "NOMEM", "NOCONV", "SOLVER", "HIP", "STATE"]
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
DIRS = {"L": 0, "R": 1, "U": 2, "D": 3, "SWEEP": 4}
INIT = {"trivial": 0, "diag": 1}

EXPORTS = [
    "ctm_config_default", "ctm_workspace_size", "ctm_init", "ctm_move", "ctm_converge",
    "ctm_spectra", "ctm_set_corner_spectra", "ctm_norm", "ctm_rdm", "ctm_rdm_complex", "ctm_expect", "ctm_fidelity",
    "ctm_env_bytes",
    "ctm_env_export", "ctm_env_import", "ctm_checkpoint_bytes", "ctm_checkpoint_save",
    "ctm_checkpoint_load", "ctm_set_metrics", "ctm_set_timing", "ctm_get_timing", "ctm_destroy",
    "ctm_last_error", "ctm_tile_table_load", "ctm_tile_table_save", "ctm_tile_table_tune",
    "ctm_tile_table_clear", "ctm_su_workspace_size", "ctm_su_init", "ctm_su_set_gates", "ctm_su_evolve",
    "ctm_su_state", "ctm_su_peps", "ctm_su_destroy", "ctm_boundary_workspace_size", "ctm_boundary_spectrum", "ctm_fidelity_noalloc", "ctm_fidelity_noalloc_max_bytes", "ctm_mlp_param_count", "ctm_mlp_workspace_size", "ctm_mlp_features",
    "ctm_mlp_targets", "ctm_mlp_forward", "ctm_mlp_loss_grad", "ctm_mlp_adam", "ctm_mlp_train",
]


class CtmConfig(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32), ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("n_tensors", ctypes.c_int32),
        ("pattern", ctypes.POINTER(ctypes.c_int32)), ("d", ctypes.POINTER(ctypes.c_int32)),
        ("D", ctypes.POINTER(ctypes.c_int32)), ("chi", ctypes.POINTER(ctypes.c_int32)),
        ("prec", ctypes.c_int32), ("svd_oversample", ctypes.c_int32),
        ("svd_max_iters", ctypes.c_int32), ("svd_resid_tol", ctypes.c_double),
        ("svd_cutoff", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
        ("concurrent_classes", ctypes.c_int32), ("single_layer", ctypes.c_int32),
        ("complex_tensors", ctypes.c_int32),
    ]


class MlpShape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32)]


class CtmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ctm status %s: %s" % (STATUS_NAMES[status] if 0 <= status < 8 else status, msg))
        self.status = status


_lib = None


def load(path=LIB_PATH, tile_table=True):
    """Load libctm.so (raises if it has not been built) and, with tile_table,
    the committed launch-variant table."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libctm.so not built (run __graft_entry__.build()): %s" % path)
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes the library bind to that runtime, so that torch's device pointers
    # and streams are valid in library calls
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, F64, SZ, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
    cfgp = P(CtmConfig)
    dpp = P(ctypes.c_void_p)
    lib.ctm_config_default.argtypes = [cfgp]
    lib.ctm_config_default.restype = None
    lib.ctm_workspace_size.argtypes = [cfgp, P(SZ)]
    lib.ctm_init.argtypes = [cfgp, dpp, dpp, VP, SZ, VP, I32, P(F64), P(VP)]
    lib.ctm_move.argtypes = [VP, I32, I32]
    lib.ctm_converge.argtypes = [VP, F64, I32, I32, P(I32), P(F64)]
    lib.ctm_spectra.argtypes = [VP, I32, P(F64)]
    lib.ctm_norm.argtypes = [VP, I32, P(F64)]
    lib.ctm_set_corner_spectra.argtypes = [VP, I32, P(F64)]
    lib.ctm_set_corner_spectra.restype = ctypes.c_int
    lib.ctm_rdm.argtypes = [VP, I32, I32, I32, I32, P(F64), P(F64)]
    lib.ctm_rdm_complex.argtypes = [VP, I32, I32, I32, I32, P(F64), P(F64)]
    lib.ctm_expect.argtypes = [VP, I32, I32, I32, I32, P(F64), P(F64)]
    lib.ctm_fidelity.argtypes = [cfgp, dpp, dpp, VP, SZ, VP, F64, I32, P(F64), P(F64), P(I32)]
    lib.ctm_boundary_workspace_size.argtypes = [VP, I32, I32, I32, P(SZ)]
    lib.ctm_boundary_workspace_size.restype = ctypes.c_int
    lib.ctm_boundary_spectrum.argtypes = [VP, I32, I32, I32, I32, I32, ctypes.c_uint64, VP, SZ, I32, P(F64), P(F64),
                                          P(F64), P(F64)]
    lib.ctm_boundary_spectrum.restype = ctypes.c_int
    lib.ctm_fidelity_noalloc.argtypes = [cfgp, dpp, dpp, VP, F64, I32, P(F64), P(F64), P(I32)]
    lib.ctm_fidelity_noalloc.restype = ctypes.c_int
    lib.ctm_fidelity_noalloc_max_bytes.argtypes = []
    lib.ctm_fidelity_noalloc_max_bytes.restype = SZ
    lib.ctm_env_bytes.argtypes = [VP, I32]
    lib.ctm_env_bytes.restype = SZ
    lib.ctm_env_export.argtypes = [VP, I32, VP, SZ]
    lib.ctm_env_import.argtypes = [VP, I32, VP, SZ]
    lib.ctm_checkpoint_bytes.argtypes = [VP, I32]
    lib.ctm_checkpoint_bytes.restype = SZ
    lib.ctm_checkpoint_save.argtypes = [VP, I32, VP, SZ]
    lib.ctm_checkpoint_load.argtypes = [VP, I32, VP, SZ]
    lib.ctm_su_workspace_size.argtypes = [I32, I32, I32, P(SZ)]
    lib.ctm_su_init.argtypes = [I32, I32, I32, VP, VP, VP, SZ, VP, P(VP)]
    lib.ctm_su_set_gates.argtypes = [VP, VP, F64]
    lib.ctm_su_evolve.argtypes = [VP, I32, F64, I32, P(I32), P(F64)]
    lib.ctm_su_state.argtypes = [VP, VP, VP]
    lib.ctm_su_peps.argtypes = [VP, VP]
    lib.ctm_su_destroy.argtypes = [VP]
    lib.ctm_su_destroy.restype = None
    for name in ("ctm_su_workspace_size", "ctm_su_init", "ctm_su_set_gates", "ctm_su_evolve", "ctm_su_state",
                 "ctm_su_peps"):
        getattr(lib, name).restype = ctypes.c_int
    lib.ctm_set_metrics.argtypes = [VP, ctypes.c_char_p, I32]
    lib.ctm_set_metrics.restype = ctypes.c_int
    lib.ctm_set_timing.argtypes = [VP, I32]
    lib.ctm_get_timing.argtypes = [VP, P(F64)]
    lib.ctm_destroy.argtypes = [VP]
    lib.ctm_destroy.restype = None
    lib.ctm_last_error.argtypes = []
    lib.ctm_last_error.restype = ctypes.c_char_p
    shp = P(MlpShape)
    lib.ctm_mlp_param_count.argtypes = [shp]
    lib.ctm_mlp_param_count.restype = ctypes.c_int64
    lib.ctm_mlp_workspace_size.argtypes = [shp, I32, P(SZ)]
    lib.ctm_mlp_features.argtypes = [VP, I32, VP, VP]
    lib.ctm_mlp_targets.argtypes = [VP, ctypes.c_int64, F64, VP, VP]
    lib.ctm_mlp_forward.argtypes = [shp, VP, VP, I32, VP, I32, VP, SZ, VP]
    lib.ctm_mlp_loss_grad.argtypes = [shp, VP, VP, VP, I32, VP, VP, VP, SZ, VP]
    lib.ctm_mlp_adam.argtypes = [ctypes.c_int64, VP, VP, VP, VP, I32, F64, F64, F64, F64, VP]
    lib.ctm_mlp_train.argtypes = [shp, VP, VP, VP, VP, I32, VP, VP, I32, I32, F64, VP, VP, SZ, VP]
    for name in ("ctm_mlp_workspace_size", "ctm_mlp_features", "ctm_mlp_targets", "ctm_mlp_forward",
                 "ctm_mlp_loss_grad", "ctm_mlp_adam", "ctm_mlp_train"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("ctm_tile_table_load", "ctm_tile_table_save"):
        getattr(lib, name).argtypes = [ctypes.c_char_p, P(I32)]
        getattr(lib, name).restype = ctypes.c_int
    lib.ctm_tile_table_tune.argtypes = [I32]
    lib.ctm_tile_table_tune.restype = ctypes.c_int
    lib.ctm_tile_table_clear.argtypes = []
    lib.ctm_tile_table_clear.restype = ctypes.c_int
    for name in ("ctm_workspace_size", "ctm_init", "ctm_move", "ctm_converge", "ctm_spectra",
                 "ctm_norm", "ctm_rdm", "ctm_rdm_complex", "ctm_expect", "ctm_fidelity", "ctm_env_export",
                 "ctm_env_import", "ctm_checkpoint_save", "ctm_checkpoint_load", "ctm_set_timing",
                 "ctm_get_timing"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    if tile_table and os.path.exists(TILE_TABLE):
        n = ctypes.c_int32()
        _check(lib.ctm_tile_table_load(TILE_TABLE.encode(), ctypes.byref(n)))
    return lib


def _check(st, allow=()):
    if st != CTM_OK and st not in allow:
        raise CtmError(st, _lib.ctm_last_error().decode())
    return st


def _i32arr(v):
    return (ctypes.c_int32 * len(v))(*[int(t) for t in v])


def make_config(Lx, Ly, pattern, n_tensors, d, D, chi, prec="fp64", oversample=16,
                max_iters=30, resid_tol=1e-13, cutoff=1e-12, seed=12345, use_graph=False,
                autotune=True, concurrent_classes=True, single_layer=False, complex_tensors=False):
    """ctm_config plus the ctypes arrays it points into (keep both alive)."""
    lib = load()
    cfg = CtmConfig()
    lib.ctm_config_default(ctypes.byref(cfg))
    d, D, chi = list(d), list(D), list(chi)
    keep = [_i32arr(pattern), _i32arr(d), _i32arr(D), _i32arr(chi)]
    cfg.n_inst = len(d)
    cfg.Lx, cfg.Ly, cfg.n_tensors = Lx, Ly, n_tensors
    cfg.pattern, cfg.d, cfg.D, cfg.chi = [ctypes.cast(k, ctypes.POINTER(ctypes.c_int32)) for k in keep]
    cfg.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    cfg.svd_oversample = oversample
    cfg.svd_max_iters = max_iters
    cfg.svd_resid_tol = resid_tol
    cfg.svd_cutoff = cutoff
    cfg.seed = seed
    cfg.use_graph = int(bool(use_graph))
    cfg.autotune = int(bool(autotune))
    cfg.concurrent_classes = int(bool(concurrent_classes))
    cfg.single_layer = int(bool(single_layer))
    cfg.complex_tensors = int(bool(complex_tensors))
    return cfg, keep


def workspace_size(cfg):
    lib = load()
    n = ctypes.c_size_t(0)
    _check(lib.ctm_workspace_size(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def _dev_tensors(torch, arrays, device, cplx=False):
    # complex tensors travel as float64 (real, imaginary) pairs
    if cplx:
        arrays = [np.ascontiguousarray(a, dtype=np.complex128).view(np.float64) for a in arrays]
    ts = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device) for a in arrays]
    ptrs = (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
    return ts, ptrs


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class CTM:
    """One CTM context: `kets` is a list (instances) of lists (tensors) of
    numpy arrays [s, u, l, d, r]; `bras` the same or None."""

    def __init__(self, kets, Lx=1, Ly=1, pattern=None, chi=16, prec="fp64", bras=None,
                 init="trivial", spectrum=None, device="cuda:0", **solver):
        import torch
        self._torch = torch
        lib = load()
        if isinstance(kets[0], np.ndarray):
            kets = [kets]
            bras = [bras] if bras is not None else None
        self.n_inst = len(kets)
        nt = len(kets[0])
        if pattern is None:
            pattern = [0] * (Lx * Ly)
        chis = chi if isinstance(chi, (list, tuple)) else [chi] * self.n_inst
        d = [k[0].shape[0] for k in kets]
        D = [k[0].shape[1] for k in kets]
        self.Lx, self.Ly, self.d, self.D, self.chi = Lx, Ly, d, D, list(chis)
        # complex kets: the bra is their conjugate (no separate bras)
        self.complex = any(np.iscomplexobj(a) for inst in kets for a in inst)
        if self.complex and bras is not None:
            raise ValueError("complex kets take no bras (the bra is the conjugate of the ket)")
        self.cfg, self._keep = make_config(Lx, Ly, pattern, nt, d, D, chis, prec, complex_tensors=self.complex,
                                           **solver)
        self.device = torch.device(device)
        nbytes = workspace_size(self.cfg)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        flat_k = [a for inst in kets for a in inst]
        self._kt, kp = _dev_tensors(torch, flat_k, self.device, self.complex)
        bp = None
        if bras is not None:
            flat_b = [a for inst in bras for a in inst]
            self._bt, bp = _dev_tensors(torch, flat_b, self.device)
        sp = None
        if spectrum is not None:
            spectrum = np.ascontiguousarray(spectrum, dtype=np.float64)
            sp = spectrum.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self._spec = spectrum
        self.ctx = ctypes.c_void_p()
        if solver.get("use_graph"):
            # graph capture needs a stream of its own (not the legacy default
            # stream); the copies above ran on the current stream
            self._side = torch.cuda.Stream(self.device)
            torch.cuda.synchronize(self.device)
            self.stream = ctypes.c_void_p(self._side.cuda_stream)
        else:
            self.stream = _stream(torch, self.device)
        _check(lib.ctm_init(ctypes.byref(self.cfg), ctypes.cast(kp, ctypes.POINTER(ctypes.c_void_p)),
                            ctypes.cast(bp, ctypes.POINTER(ctypes.c_void_p)) if bp is not None else None,
                            ctypes.c_void_p(base + off), nbytes, self.stream, INIT[init], sp,
                            ctypes.byref(self.ctx)))

    def move(self, direction, count=1):
        _check(load().ctm_move(self.ctx, DIRS[direction] if isinstance(direction, str) else direction, count))

    def sweep(self, count=1):
        self.move("SWEEP", count)

    def converge(self, tol=1e-10, max_sweeps=500, check_every=1):
        n = self.n_inst
        sw = (ctypes.c_int32 * n)()
        dl = (ctypes.c_double * n)()
        st = _check(load().ctm_converge(self.ctx, tol, max_sweeps, check_every, sw, dl), allow=(CTM_E_NOCONV,))
        return list(sw), list(dl), st == CTM_OK

    def spectra(self, inst=0):
        out = np.zeros((self.Lx * self.Ly, 4, self.chi[inst]))
        _check(load().ctm_spectra(self.ctx, inst, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_corner_spectra(self, spectra, inst=0):
        """New singular values [Lx*Ly, 4, chi] for every corner, vectors kept."""
        sp = np.ascontiguousarray(spectra, dtype=np.float64).reshape(self.Lx * self.Ly, 4, self.chi[inst])
        _check(load().ctm_set_corner_spectra(self.ctx, inst, sp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def norm(self, inst=0):
        v = ctypes.c_double()
        _check(load().ctm_norm(self.ctx, inst, ctypes.byref(v)))
        return v.value

    def rdm(self, x, y, vertical=False, inst=0):
        """(rho, hermiticity defect); rho complex for complex kets."""
        m = self.d[inst] ** 2
        h = ctypes.c_double()
        if self.complex:
            out = np.zeros((m, m), dtype=np.complex128)
            _check(load().ctm_rdm_complex(self.ctx, inst, x, y, int(vertical),
                                          out.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.byref(h)))
            return out, h.value
        out = np.zeros((m, m))
        _check(load().ctm_rdm(self.ctx, inst, x, y, int(vertical),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)))
        return out, h.value

    def expect(self, x, y, vertical, op, inst=0):
        op = np.ascontiguousarray(np.real(op), dtype=np.float64)
        v = ctypes.c_double()
        _check(load().ctm_expect(self.ctx, inst, x, y, int(vertical),
                                 op.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(v)))
        return v.value

    def export_env(self, inst=0):
        n = load().ctm_env_bytes(self.ctx, inst)
        buf = np.zeros(n // 8)
        _check(load().ctm_env_export(self.ctx, inst, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def import_env(self, buf, inst=0):
        buf = np.ascontiguousarray(buf, dtype=np.float64)
        _check(load().ctm_env_import(self.ctx, inst, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))

    def save_checkpoint(self, inst=0):
        """Everything the next sweeps depend on (ctm_checkpoint_save), as bytes."""
        n = load().ctm_checkpoint_bytes(self.ctx, inst)
        buf = np.zeros(n, dtype=np.uint8)
        _check(load().ctm_checkpoint_save(self.ctx, inst, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def load_checkpoint(self, buf, inst=0):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(load().ctm_checkpoint_load(self.ctx, inst, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))

    def boundary_spectrum(self, nv, column=0, krylov=None, block=4, nev=None, seed=7, inst=0):
        """Leading eigenvalues of sigma_L^T sigma_R on an nv cylinder divided by
        the trace (ctm_boundary_spectrum): (eigenvalues, residuals, entropy,
        captured weight)."""
        lib = load()
        dim = self.D[inst] ** nv
        krylov = dim if krylov is None else krylov
        nev = krylov if nev is None else nev
        nb = ctypes.c_size_t()
        _check(lib.ctm_boundary_workspace_size(self.ctx, inst, nv, krylov, ctypes.byref(nb)))
        ws = self._torch.empty(nb.value + 256, dtype=self._torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        ev = np.zeros(nev)
        res = np.zeros(nev)
        ent, wt = ctypes.c_double(), ctypes.c_double()
        P = ctypes.POINTER(ctypes.c_double)
        _check(lib.ctm_boundary_spectrum(self.ctx, inst, column, nv, krylov, block, seed,
                                         ctypes.c_void_p(ws.data_ptr() + off), nb.value, nev,
                                         ev.ctypes.data_as(P), res.ctypes.data_as(P), ctypes.byref(ent),
                                         ctypes.byref(wt)))
        self._torch.cuda.synchronize(self.device)
        del ws
        return ev, res, ent.value, wt.value

    def set_metrics(self, path, kappa=False):
        """Per-check JSON metrics lines of converge appended to `path` ("-":
        standard error, None: off); kappa adds the norm per site to each
        line (ctm_set_metrics)."""
        _check(load().ctm_set_metrics(self.ctx, None if path is None else str(path).encode(), 1 if kappa else 0))

    def set_timing(self, mode=1):
        """1: phases and corner-kernel launches, 2: corner-kernel launches
        only, 0 / False: off (see ctm_set_timing)."""
        _check(load().ctm_set_timing(self.ctx, int(mode)))

    def timing(self):
        v = (ctypes.c_double * 10)()
        _check(load().ctm_get_timing(self.ctx, v))
        keys = ["corner_s", "solver_s", "absorb_s", "stage3_s", "stage3_launches", "stage3_flop",
                "corner_launches", "moves", "stage3_flop_nominal", "live_chi"]
        return dict(zip(keys, list(v)))

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self._torch.cuda.synchronize(self.device)
            load().ctm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fidelity(A_list, B_list, Lx=1, Ly=1, pattern=None, chi=16, prec="fp64", tol=1e-10,
             max_sweeps=200, device="cuda:0", **solver):
    """Fidelity per site between the states of two tensor sets: (d, ln d,
    sweeps of the three CTM runs, whether all three converged)."""
    import torch
    lib = load()
    if any(np.iscomplexobj(a) for a in list(A_list) + list(B_list)):
        raise ValueError("fidelity needs real tensors (the mixed network of complex states has no real form)")
    if pattern is None:
        pattern = [0] * (Lx * Ly)
    d = [A_list[0].shape[0]]
    D = [A_list[0].shape[1]]
    cfg, keep = make_config(Lx, Ly, pattern, len(A_list), d, D, [chi], prec, **solver)
    dev = torch.device(device)
    nbytes = workspace_size(cfg)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    at, ap = _dev_tensors(torch, A_list, dev)
    bt, bp = _dev_tensors(torch, B_list, dev)
    dv, lv = ctypes.c_double(), ctypes.c_double()
    sw = (ctypes.c_int32 * 3)()
    st = _check(lib.ctm_fidelity(ctypes.byref(cfg), ctypes.cast(ap, ctypes.POINTER(ctypes.c_void_p)),
                                 ctypes.cast(bp, ctypes.POINTER(ctypes.c_void_p)),
                                 ctypes.c_void_p(ws.data_ptr() + off), nbytes, _stream(torch, dev), tol,
                                 max_sweeps, ctypes.byref(dv), ctypes.byref(lv), sw), allow=(CTM_E_NOCONV,))
    torch.cuda.synchronize(dev)
    del at, bt, ws
    return dv.value, lv.value, list(sw), st == CTM_OK


def fidelity_noalloc(A_list, B_list, Lx=1, Ly=1, pattern=None, chi=16, prec="fp64", tol=1e-10,
                     max_sweeps=200, device="cuda:0", **solver):
    """As fidelity(), through ctm_fidelity_noalloc: the library allocates
    nothing (its workspace is a static device array); only the tensor copies
    are made here."""
    import torch
    lib = load()
    if any(np.iscomplexobj(a) for a in list(A_list) + list(B_list)):
        raise ValueError("fidelity needs real tensors (the mixed network of complex states has no real form)")
    if pattern is None:
        pattern = [0] * (Lx * Ly)
    cfg, keep = make_config(Lx, Ly, pattern, len(A_list), [A_list[0].shape[0]], [A_list[0].shape[1]], [chi],
                            prec, **solver)
    dev = torch.device(device)
    at, ap = _dev_tensors(torch, A_list, dev)
    bt, bp = _dev_tensors(torch, B_list, dev)
    dv, lv = ctypes.c_double(), ctypes.c_double()
    sw = (ctypes.c_int32 * 3)()
    st = _check(lib.ctm_fidelity_noalloc(ctypes.byref(cfg), ctypes.cast(ap, ctypes.POINTER(ctypes.c_void_p)),
                                         ctypes.cast(bp, ctypes.POINTER(ctypes.c_void_p)), _stream(torch, dev),
                                         tol, max_sweeps, ctypes.byref(dv), ctypes.byref(lv), sw),
                allow=(CTM_E_NOCONV,))
    torch.cuda.synchronize(dev)
    del at, bt
    return dv.value, lv.value, list(sw), st == CTM_OK


class MLP:
    """Warm-start network on the device (include/ctm_mlp.h): float64 parameters,
    Adam moments and workspace held as torch tensors; every computation is a
    library call."""

    def __init__(self, n_in, n_hidden, n_out, params, max_batch, device="cuda:0"):
        import torch
        self._torch = torch
        lib = load()
        self.shape = MlpShape(n_in, n_hidden, n_out)
        self.n_params = lib.ctm_mlp_param_count(ctypes.byref(self.shape))
        if self.n_params < 0:
            raise CtmError(CTM_E_INVALID, "bad network shape")
        params = np.ascontiguousarray(params, dtype=np.float64)
        if params.size != self.n_params:
            raise CtmError(CTM_E_INVALID, "expected %d parameters" % self.n_params)
        self.device = torch.device(device)
        self.p = torch.as_tensor(params, device=self.device).clone()
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.step = 0
        self.max_batch = max_batch
        nb = ctypes.c_size_t()
        _check(lib.ctm_mlp_workspace_size(ctypes.byref(self.shape), max_batch, ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        self._off = (-self._ws.data_ptr()) % 256
        self.ws_bytes = nb.value
        self.stream = _stream(torch, self.device)

    def _ws_ptr(self):
        return ctypes.c_void_p(self._ws.data_ptr() + self._off)

    def _dev(self, a):
        return self._torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr())

    def features(self, theta):
        th = self._dev(theta)
        x = self._torch.empty((th.shape[0], 3), dtype=self._torch.float64, device=self.device)
        _check(load().ctm_mlp_features(self._ptr(th), th.shape[0], self._ptr(x), self.stream))
        return x

    def targets(self, spectra, floor=1e-16):
        s = self._dev(spectra)
        t = self._torch.empty_like(s)
        _check(load().ctm_mlp_targets(self._ptr(s), s.numel(), floor, self._ptr(t), self.stream))
        return t.reshape(s.shape[0], -1)

    def forward(self, x, exp10=False):
        B = x.shape[0]
        y = self._torch.empty((B, self.shape.n_out), dtype=self._torch.float64, device=self.device)
        _check(load().ctm_mlp_forward(ctypes.byref(self.shape), self._ptr(self.p), self._ptr(x), B, self._ptr(y),
                                      int(exp10), self._ws_ptr(), self.ws_bytes, self.stream))
        return y

    def loss_grad(self, x, t):
        _check(load().ctm_mlp_loss_grad(ctypes.byref(self.shape), self._ptr(self.p), self._ptr(x), self._ptr(t),
                                        x.shape[0], self._ptr(self.loss_dev), self._ptr(self.g), self._ws_ptr(),
                                        self.ws_bytes, self.stream))
        return float(self.loss_dev.item()), self.g.clone()

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(load().ctm_mlp_adam(self.n_params, self._ptr(self.p), self._ptr(self.g), self._ptr(self.m),
                                   self._ptr(self.v), self.step, lr, beta1, beta2, eps, self.stream))

    def train(self, x, t, steps, lr):
        hist = self._torch.zeros(max(steps, 1), dtype=self._torch.float64, device=self.device)
        _check(load().ctm_mlp_train(ctypes.byref(self.shape), self._ptr(self.p), self._ptr(self.m),
                                    self._ptr(self.v), self._ptr(self.g), self.step, self._ptr(x), self._ptr(t),
                                    x.shape[0], steps, lr, self._ptr(hist), self._ws_ptr(), self.ws_bytes,
                                    self.stream))
        self.step += steps
        return hist[:steps].cpu().numpy()


class SimpleUpdate:
    """Simple update of n 2x2-checkerboard states in lock-step (ctm_su_*).
    `tensors`: n pairs (A, B) of numpy arrays [s, u, l, d, r] (the Gamma
    tensors); `weights`: array [n][4][D] over the bonds h0, h1, v0, v1."""

    def __init__(self, tensors, weights, device="cuda:0"):
        import torch
        self._torch = torch
        lib = load()
        self.device = torch.device(device)
        self.n = len(tensors)
        self.d, self.D = int(tensors[0][0].shape[0]), int(tensors[0][0].shape[1])
        T = np.ascontiguousarray(np.stack([np.stack(inst) for inst in tensors]), dtype=np.float64)
        L = np.ascontiguousarray(weights, dtype=np.float64)
        assert T.shape == (self.n, 2, self.d) + (self.D,) * 4 and L.shape == (self.n, 4, self.D)
        tT = torch.as_tensor(T, device=self.device)
        tL = torch.as_tensor(L, device=self.device)
        nb = ctypes.c_size_t()
        _check(lib.ctm_su_workspace_size(self.n, self.d, self.D, ctypes.byref(nb)))
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.stream = _stream(torch, self.device)
        self.ctx = ctypes.c_void_p()
        _check(lib.ctm_su_init(self.n, self.d, self.D, ctypes.c_void_p(tT.data_ptr()), ctypes.c_void_p(tL.data_ptr()),
                               ctypes.c_void_p(self.ws.data_ptr() + off), nb.value, self.stream,
                               ctypes.byref(self.ctx)))
        torch.cuda.synchronize(self.device)

    def set_gates(self, h, dtau):
        """Gates exp(-dtau h) from bond Hamiltonians h [n][4][d^2][d^2]."""
        th = self._torch.as_tensor(np.ascontiguousarray(h, dtype=np.float64), device=self.device)
        _check(load().ctm_su_set_gates(self.ctx, ctypes.c_void_p(th.data_ptr()), float(dtau)))

    def evolve(self, max_steps, tol=0.0, check_every=10):
        """Trotter steps (ctm_su_evolve): (steps done, last weight change per instance)."""
        steps = ctypes.c_int32()
        ch = (ctypes.c_double * self.n)()
        _check(load().ctm_su_evolve(self.ctx, int(max_steps), float(tol), int(check_every), ctypes.byref(steps), ch))
        return steps.value, np.array(ch[:])

    def state(self):
        """(Gamma tensors [n][2][d, D, D, D, D], weights [n][4][D])."""
        torch = self._torch
        T = torch.empty((self.n, 2, self.d) + (self.D,) * 4, dtype=torch.float64, device=self.device)
        L = torch.empty((self.n, 4, self.D), dtype=torch.float64, device=self.device)
        _check(load().ctm_su_state(self.ctx, ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(L.data_ptr())))
        return T.cpu().numpy(), L.cpu().numpy()

    def peps(self):
        """iPEPS tensors with sqrt(weights) on every leg [n][2][d, D, D, D, D]."""
        torch = self._torch
        T = torch.empty((self.n, 2, self.d) + (self.D,) * 4, dtype=torch.float64, device=self.device)
        _check(load().ctm_su_peps(self.ctx, ctypes.c_void_p(T.data_ptr())))
        return T.cpu().numpy()

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self._torch.cuda.synchronize(self.device)
            load().ctm_su_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
