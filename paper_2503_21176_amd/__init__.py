"""Python binding of libpmeqeq: periodic Coulomb (Ewald / smooth PME) and
charge equilibration on AMD MI355X.

Argument marshalling only: every step runs in the HIP library behind the C
ABI declared in include/pmeqeq.h. Tensors are torch CUDA (HIP) tensors,
float64, contiguous, on the context's device; PyTorch provides device memory
and the current stream. If the library is not built, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmeqeq.so")

ABI_VERSION = 5
PQ_OK = 0
FLAG_FP64 = 1
FLAG_COMPENSATED = 2
PQ_WARN_NOT_CONVERGED = 1
STATUS = {0: "PQ_OK", 1: "PQ_WARN_NOT_CONVERGED", -1: "PQ_ERR_INVALID", -2: "PQ_ERR_BOX",
          -3: "PQ_ERR_CAPACITY", -4: "PQ_ERR_NOMEM", -5: "PQ_ERR_HIP", -6: "PQ_ERR_TOO_LARGE",
          -7: "PQ_ERR_NAN", -8: "PQ_ERR_STATE", -9: "PQ_ERR_TIMEOUT"}
METHOD_PME, METHOD_EWALD, METHOD_AUTO = 0, 1, 2
SOLVERS = {"gmres": 0, "minres": 1}

EXPORTS = ["pq_abi_version", "pq_coulomb_constant", "pq_last_error", "pq_ctx_last_error", "pq_create", "pq_set_stream",
           "pq_destroy", "pq_set_system", "pq_neighbor_pairs", "pq_coulomb", "pq_set_timing", "pq_timings",
           "pq_qeq_solve", "pq_shadow_step", "pq_qeq_vjp", "pq_server_create", "pq_server_submit",
           "pq_server_poll", "pq_server_destroy", "pq_request_footprint", "pq_autotune", "pq_set_tuning",
           "pq_choose_params", "pq_auto_pme_min_atoms", "pq_md_run", "pq_md_history", "pq_coulomb_noalloc",
           "pq_set_solver", "pq_update_positions", "pq_neighbor_ell"]
PHASES = ["stage", "pair", "spread", "fft", "gather", "combine", "total"]


class PQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("cutoff", ctypes.c_double), ("skin", ctypes.c_double),
                ("alpha", ctypes.c_double), ("grid", ctypes.c_int32 * 3), ("order", ctypes.c_int32),
                ("kmax", ctypes.c_int32 * 3), ("method", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tilt", ctypes.c_double * 3)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("lambda_", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("pair_wg_per_cu", ctypes.c_int32), ("candidates", ctypes.c_int32), ("ms", ctypes.c_double),
                ("ms_default", ctypes.c_double), ("fft_lds_bytes", ctypes.c_int32), ("pair_fork", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user_data", ctypes.c_void_p)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("pos", ctypes.c_void_p), ("chi", ctypes.c_void_p),
                ("eta", ctypes.c_void_p), ("q0", ctypes.c_void_p), ("q_tot", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_it", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("reserved", ctypes.c_int32), ("params", Params)]


class Result(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p), ("energy", ctypes.c_double), ("info", SolveInfo),
                ("status", ctypes.c_int32), ("t_submit_s", ctypes.c_double), ("t_start_s", ctypes.c_double),
                ("t_done_s", ctypes.c_double), ("message", ctypes.c_char * 256)]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libpmeqeq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_21176_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    sig = {
        "pq_abi_version": (i32, []),
        "pq_coulomb_constant": (dbl, []),
        "pq_last_error": (ctypes.c_char_p, []),
        "pq_ctx_last_error": (ctypes.c_char_p, [vp]),
        "pq_create": (i32, [ctypes.POINTER(vp), i32, vp, ctypes.POINTER(Allocator)]),
        "pq_set_stream": (i32, [vp, vp]),
        "pq_destroy": (i32, [vp]),
        "pq_set_system": (i32, [vp, i64, vp, ctypes.POINTER(Params)]),
        "pq_neighbor_pairs": (i32, [vp, i64, vp, ctypes.POINTER(i64)]),
        "pq_neighbor_ell": (i32, [vp, i32, vp, vp, vp, ctypes.POINTER(i32)]),
        "pq_coulomb": (i32, [vp, vp, vp, vp, vp]),
        "pq_coulomb_noalloc": (i32, [vp, vp, vp, vp, vp]),
        "pq_set_solver": (i32, [vp, i32, i32]),
        "pq_update_positions": (i32, [vp, vp, ctypes.POINTER(i32)]),
        "pq_set_timing": (i32, [vp, i32]),
        "pq_timings": (i32, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "pq_qeq_solve": (i32, [vp, vp, vp, dbl, dbl, i32, i32, vp, vp, vp, vp, ctypes.POINTER(SolveInfo)]),
        "pq_shadow_step": (i32, [vp, vp, vp, dbl, vp, i32, vp, vp, vp, vp]),
        "pq_qeq_vjp": (i32, [vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp]),
        "pq_server_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(ServerCfg)]),
        "pq_server_submit": (i32, [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
        "pq_server_poll": (i32, [vp, ctypes.c_uint64, ctypes.POINTER(Result), i64]),
        "pq_server_destroy": (i32, [vp]),
        "pq_request_footprint": (dbl, [i64, ctypes.POINTER(Params), i32]),
        "pq_autotune": (i32, [vp, vp, i32, ctypes.POINTER(TuneResult)]),
        "pq_set_tuning": (i32, [vp, ctypes.POINTER(TuneResult)]),
        "pq_choose_params": (i32, [ctypes.POINTER(dbl), i64, dbl, dbl, i32, i32, ctypes.POINTER(Params)]),
        "pq_auto_pme_min_atoms": (i64, []),
        "pq_md_run": (i32, [vp, vp, vp, vp, vp, vp, dbl, vp, vp, i32, ctypes.POINTER(MdCfg), vp]),
        "pq_md_history": (i32, [i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    if L.pq_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {L.pq_abi_version()}, the binding expects {ABI_VERSION}")
    _lib = L
    return L


def _check(code: int, allow_warn: bool = False) -> int:
    if code == PQ_OK or (allow_warn and code == PQ_WARN_NOT_CONVERGED):
        return code
    raise PQError(code, load().pq_last_error().decode(errors="replace"))


def coulomb_constant() -> float:
    return float(load().pq_coulomb_constant())


def make_params(box, cutoff, alpha, skin=0.0, grid=None, order=6, kmax=None, method="pme",
                fp64=False, compensated=False) -> Params:
    """Parameters of one periodic system. ``box``: an edge, three edges, or a
    3x3 lower triangular matrix whose rows are the lattice vectors
    a = (L0, 0, 0), b = (t_xy, L1, 0), c = (t_xz, t_yz, L2) (triclinic).
    ``fp64`` selects FP64 bulk arithmetic (PQ_FLAG_FP64) instead of the
    default FP32 bulk with FP64 reductions; ``compensated`` the compensated
    FP32 pair sums (PQ_FLAG_COMPENSATED)."""
    p = Params()
    H = np.asarray(box, np.float64)
    if H.shape == (3, 3):
        if H[0, 1] != 0 or H[0, 2] != 0 or H[1, 2] != 0:
            raise ValueError("a triclinic box must be lower triangular (rows a, b, c)")
        p.box[:] = [float(H[0, 0]), float(H[1, 1]), float(H[2, 2])]
        p.tilt[:] = [float(H[1, 0]), float(H[2, 0]), float(H[2, 1])]
    else:
        b = [float(x) for x in (box if hasattr(box, "__len__") else (box, box, box))]
        p.box[:] = b
    p.cutoff, p.skin, p.alpha = float(cutoff), float(skin), float(alpha)
    if method == "pme":
        g = grid if hasattr(grid, "__len__") else (grid, grid, grid)
        p.grid[:] = [int(x) for x in g]
        p.order = int(order)
        p.method = METHOD_PME
    elif method == "ewald":
        k = kmax if hasattr(kmax, "__len__") else (kmax, kmax, kmax)
        p.kmax[:] = [int(x) for x in k]
        p.method = METHOD_EWALD
    else:
        raise ValueError(method)
    p.flags = (FLAG_FP64 if fp64 else 0) | (FLAG_COMPENSATED if compensated else 0)
    return p


class MdCfg(ctypes.Structure):
    _fields_ = [("dt_fs", ctypes.c_double), ("n_krylov", ctypes.c_int32), ("dissipation", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("rep_a", ctypes.c_double), ("rep_rho", ctypes.c_double),
                ("mode", ctypes.c_int32), ("max_it", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tol", ctypes.c_double)]


MD_SHADOW, MD_REGULAR = 0, 1


def md_history(dissipation: int) -> int:
    """Number of n vectors the shadow-MD driver keeps (newest first)."""
    return int(load().pq_md_history(int(dissipation)))


def md_state_save(path, pos, vel, n_hist, pos_ref):
    """Writes the state of an MD run (positions, velocities, extended-charge
    history, positions of the last full neighbour build) to a .npz file; a
    run continued from md_state_load in a fresh context with the same
    parameters repeats the uninterrupted run bit for bit."""
    np.savez(path, pos=pos.detach().cpu().numpy(), vel=vel.detach().cpu().numpy(),
             n_hist=n_hist.detach().cpu().numpy(), pos_ref=pos_ref.detach().cpu().numpy())


def md_state_load(path, device=0):
    """The state md_state_save wrote, as FP64 tensors on `device`:
    (pos, vel, n_hist, pos_ref)."""
    with np.load(path, allow_pickle=False) as z:
        dev = torch.device("cuda", device)
        return tuple(torch.as_tensor(np.ascontiguousarray(z[k]), dtype=torch.float64, device=dev)
                     for k in ("pos", "vel", "n_hist", "pos_ref"))


def choose_params(box, n, cutoff, delta=5e-4, order=6, method="auto", fp64=False) -> Params:
    """Accuracy-driven parameters (pq_choose_params): alpha, the PME grid and
    the direct-Ewald range from the target accuracy delta; ``method`` is
    "pme", "ewald" or "auto" (by atom count)."""
    m = {"pme": METHOD_PME, "ewald": METHOD_EWALD, "auto": METHOD_AUTO}[method]
    b = (ctypes.c_double * 3)(*[float(x) for x in (box if hasattr(box, "__len__") else (box, box, box))])
    p = Params()
    _check(load().pq_choose_params(b, int(n), float(cutoff), float(delta), int(order), m, ctypes.byref(p)))
    if fp64:
        p.flags = FLAG_FP64
    return p


def auto_pme_min_atoms() -> int:
    return int(load().pq_auto_pme_min_atoms())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class QeqResult:
    q: torch.Tensor
    force: torch.Tensor | None
    energy: torch.Tensor | None
    iterations: int
    restarts: int
    rel_residual: float
    lam: float
    status: int


def _torch_allocator(device: torch.device) -> Allocator:
    """The library's workspaces from torch's caching allocator (on the
    stream that is current when a block is taken)."""

    def alloc(nbytes, _ud):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, torch.cuda.current_stream(device))
        except Exception:  # out of memory: the library reports PQ_ERR_NOMEM
            return None

    def free(ptr, _ud):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:  # interpreter shutdown: torch's allocator is gone with the process
            pass

    return Allocator(ALLOC_FN(alloc), FREE_FN(free), None)


class Context:
    """One system on one device; calls are ordered on torch's current stream.
    Workspaces come from torch's caching allocator (allocator="torch") or
    from hipMalloc (allocator=None)."""

    def __init__(self, device: int = 0, allocator: str | None = "torch"):
        self.lib = load()
        self.device = torch.device("cuda", device)
        self._alloc = _torch_allocator(self.device) if allocator == "torch" else None
        h = ctypes.c_void_p()
        _check(self.lib.pq_create(ctypes.byref(h), device, None,
                                  ctypes.byref(self._alloc) if self._alloc is not None else None))
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.pq_destroy(self.h)
            self.h = None

    def last_error(self) -> str:
        """Message of the last failed call on this context ("" if none)."""
        return self.lib.pq_ctx_last_error(self.h).decode() if getattr(self, "h", None) else ""

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib.pq_set_stream(self.h, ctypes.c_void_p(s)))

    def _vec(self, t, n, name, cols=None):
        if t is None:
            return None
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        shape = (n,) if cols is None else (n, cols)
        if n > 0 and tuple(t.shape) != shape:   # n == 0: no system; the library reports it
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, context is on {self.device}")
        return t.contiguous()

    def set_system(self, pos: torch.Tensor, params: Params):
        n = int(pos.shape[0])
        pos = self._vec(pos, n, "pos", 3)
        self._sync_stream()
        _check(self.lib.pq_set_system(self.h, n, _ptr(pos), ctypes.byref(params)))
        self.n, self.params = n, params

    def update_positions(self, pos: torch.Tensor) -> bool:
        """Moves the atoms, keeping the neighbour list while every atom is
        within skin/2 of its last build position; returns True if it rebuilt."""
        pos = self._vec(pos, self.n, "pos", 3)
        r = ctypes.c_int32()
        self._sync_stream()
        _check(self.lib.pq_update_positions(self.h, _ptr(pos), ctypes.byref(r)))
        return bool(r.value)

    def neighbor_count(self) -> int:
        cnt = ctypes.c_int64()
        self._sync_stream()
        _check(self.lib.pq_neighbor_pairs(self.h, 0, None, ctypes.byref(cnt)))
        return int(cnt.value)

    def neighbor_pairs(self) -> torch.Tensor:
        cnt = ctypes.c_int64()
        self._sync_stream()
        _check(self.lib.pq_neighbor_pairs(self.h, 0, None, ctypes.byref(cnt)))
        out = torch.empty((max(1, cnt.value), 5), dtype=torch.int32, device=self.device)
        _check(self.lib.pq_neighbor_pairs(self.h, cnt.value, _ptr(out), ctypes.byref(cnt)))
        return out[:cnt.value]

    def neighbor_ell(self, images: bool = True):
        """ELLPACK neighbour matrix (n x K, K the largest row count): rows of
        neighbour indices in ascending (j, image) order padded with -1, their
        image vectors (n x K x 3, or None) and the row counts."""
        km = ctypes.c_int32()
        cnt = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self._sync_stream()
        _check(self.lib.pq_neighbor_ell(self.h, 0, None, None, _ptr(cnt), ctypes.byref(km)))
        K = int(km.value)
        nbr = torch.empty((self.n, K), dtype=torch.int32, device=self.device)
        img = torch.empty((self.n, K, 3), dtype=torch.int32, device=self.device) if images else None
        if K:
            _check(self.lib.pq_neighbor_ell(self.h, K, _ptr(nbr), _ptr(img) if images else None, None,
                                            ctypes.byref(km)))
        return nbr, img, cnt

    def autotune(self, q, reps: int = 5) -> dict:
        """Times the pair kernel's launch shapes on phi+F evaluations with
        charges q and keeps the fastest for this context."""
        self._sync_stream()
        q = self._vec(q, self.n, "q")
        t = TuneResult()
        _check(self.lib.pq_autotune(self.h, _ptr(q), int(reps), ctypes.byref(t)))
        return dict(pair_wg_per_cu=t.pair_wg_per_cu, candidates=t.candidates, ms=t.ms, ms_default=t.ms_default,
                    fft_lds_bytes=t.fft_lds_bytes, pair_fork=t.pair_fork)

    def set_tuning(self, pair_wg_per_cu: int, fft_lds_bytes: int = 0, pair_fork: int = 0):
        t = TuneResult(int(pair_wg_per_cu), 0, 0.0, 0.0, int(fft_lds_bytes), int(pair_fork))
        _check(self.lib.pq_set_tuning(self.h, ctypes.byref(t)))

    def set_timing(self, mode=1):
        """0 off, 1 phase events (phases overlap as in production), 2 phases serialised."""
        _check(self.lib.pq_set_timing(self.h, int(mode)))

    def timings(self):
        """Per-phase device milliseconds summed since the last call, and the count."""
        ms = (ctypes.c_double * 7)()
        cnt = ctypes.c_int64()
        _check(self.lib.pq_timings(self.h, ms, ctypes.byref(cnt)))
        return dict(zip(PHASES, list(ms))), cnt.value

    def coulomb(self, q, phi=True, force=True, energy=True):
        q = self._vec(q, self.n, "q")
        o_phi = torch.empty(self.n, dtype=torch.float64, device=self.device) if phi else None
        o_f = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if force else None
        o_e = torch.empty(4, dtype=torch.float64, device=self.device) if energy else None
        self._sync_stream()
        _check(self.lib.pq_coulomb(self.h, _ptr(q), _ptr(o_phi), _ptr(o_f), _ptr(o_e)))
        return o_phi, o_f, o_e

    def coulomb_noalloc(self, q, phi, force, energy):
        """pq_coulomb_noalloc into caller-provided outputs (each FP64 device
        tensor or None: phi (n,), force (n, 3), energy (4,)); allocates nothing."""
        q = self._vec(q, self.n, "q")
        for t, shape, name in ((phi, (self.n,), "phi"), (force, (self.n, 3), "force"), (energy, (4,), "energy")):
            if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                                      and t.is_contiguous() and tuple(t.shape) == shape and t.device == self.device):
                raise ValueError(f"{name} must be a contiguous FP64 tensor of shape {shape} on {self.device}")
        self._sync_stream()
        _check(self.lib.pq_coulomb_noalloc(self.h, _ptr(q), _ptr(phi), _ptr(force), _ptr(energy)))

    def set_solver(self, solver="gmres", vjp_restart=50):
        """Krylov method of this context's QEQ solves: "gmres" (restarted,
        right Jacobi) or "minres" (preconditioned, short recurrences);
        vjp_restart is the GMRES restart length of the adjoint solve."""
        _check(self.lib.pq_set_solver(self.h, SOLVERS[solver], int(vjp_restart)))

    def qeq_solve(self, chi, eta, q_tot=0.0, tol=1e-6, max_it=500, restart=50, q0=None, force=False,
                  energy=True) -> QeqResult:
        chi, eta = self._vec(chi, self.n, "chi"), self._vec(eta, self.n, "eta")
        q0 = self._vec(q0, self.n, "q0")
        q = torch.empty(self.n, dtype=torch.float64, device=self.device)
        f = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if force else None
        e = torch.empty(1, dtype=torch.float64, device=self.device) if energy else None
        info = SolveInfo()
        self._sync_stream()
        st = _check(self.lib.pq_qeq_solve(self.h, _ptr(chi), _ptr(eta), float(q_tot), float(tol), int(max_it),
                                          int(restart), _ptr(q0), _ptr(q), _ptr(f), _ptr(e), ctypes.byref(info)),
                    allow_warn=True)
        return QeqResult(q, f, e, info.iterations, info.restarts, info.rel_residual, info.lambda_, st)

    def shadow_step(self, chi, eta, n_vec, q_tot=0.0, n_krylov=8, force=True, nddot=True, energy=True):
        chi, eta = self._vec(chi, self.n, "chi"), self._vec(eta, self.n, "eta")
        n_vec = self._vec(n_vec, self.n, "n_vec")
        dev, N = self.device, self.n
        q = torch.empty(N, dtype=torch.float64, device=dev)
        f = torch.empty((N, 3), dtype=torch.float64, device=dev) if force else None
        x = torch.empty(N, dtype=torch.float64, device=dev) if nddot else None
        e = torch.empty(2, dtype=torch.float64, device=dev) if energy else None
        self._sync_stream()
        _check(self.lib.pq_shadow_step(self.h, _ptr(chi), _ptr(eta), float(q_tot), _ptr(n_vec), int(n_krylov),
                                       _ptr(q), _ptr(f), _ptr(x), _ptr(e)))
        return q, f, x, e

    def md_run(self, pos, vel, mass, chi, eta, n_hist, steps, dt_fs=0.5, n_krylov=8, dissipation=5, kappa=1.82,
               rep_a=0.0, rep_rho=0.3, q_tot=0.0, regular=False, tol=1e-6, max_it=200, restart=50, pos_ref=None):
        """Shadow XL-BOMD steps, or regular BO-MD steps with QEQ solves to
        ``tol`` (pq_md_run). pos, vel (n x 3), n_hist (md_history(dissipation)
        x n, newest first; regular mode: row 0 the start charges) and pos_ref
        (n x 3 or None: positions of the last full neighbour build, see
        md_state) are FP64 device tensors updated in place; the context holds
        the run's parameters (pq_set_system). Returns the (steps + 1) x 6 rows
        {kinetic, potential, V_short, total (eV), Coulomb evaluations of the
        step, 1 if the neighbour list was rebuilt for the step}."""
        N = self.n
        H = md_history(dissipation)
        shapes = [(pos, (N, 3), "pos"), (vel, (N, 3), "vel"), (n_hist, (H, N), "n_hist")]
        if pos_ref is not None:
            shapes.append((pos_ref, (N, 3), "pos_ref"))
        for t, shape, name in shapes:
            if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_contiguous()
                    and tuple(t.shape) == shape and t.device == self.device):
                raise ValueError(f"{name} must be a contiguous FP64 tensor of shape {shape} on {self.device}")
        mass = self._vec(mass, N, "mass")
        chi, eta = self._vec(chi, N, "chi"), self._vec(eta, N, "eta")
        cfg = MdCfg(float(dt_fs), int(n_krylov), int(dissipation), float(kappa), float(rep_a), float(rep_rho),
                    MD_REGULAR if regular else MD_SHADOW, int(max_it), int(restart), 0, float(tol))
        e = np.zeros((int(steps) + 1, 6), dtype=np.float64)
        self._sync_stream()
        _check(self.lib.pq_md_run(self.h, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(chi), _ptr(eta), float(q_tot),
                                  _ptr(n_hist), _ptr(pos_ref), int(steps), ctypes.byref(cfg),
                                  e.ctypes.data_as(ctypes.c_void_p)))
        return e

    def qeq_vjp(self, chi, eta, q_star, gbar=None, tol=1e-8, max_it=1000, with_status=False):
        """(d_pos, d_chi, d_eta), plus the status of the adjoint solve
        (PQ_WARN_NOT_CONVERGED possible with gbar) when with_status."""
        chi, eta = self._vec(chi, self.n, "chi"), self._vec(eta, self.n, "eta")
        q_star = self._vec(q_star, self.n, "q_star")
        gbar = self._vec(gbar, self.n, "gbar")
        dev, N = self.device, self.n
        dpos = torch.empty((N, 3), dtype=torch.float64, device=dev)
        dchi = torch.empty(N, dtype=torch.float64, device=dev)
        deta = torch.empty(N, dtype=torch.float64, device=dev)
        self._sync_stream()
        st = _check(self.lib.pq_qeq_vjp(self.h, _ptr(chi), _ptr(eta), _ptr(q_star), _ptr(gbar), float(tol),
                                        int(max_it), _ptr(dpos), _ptr(dchi), _ptr(deta)), allow_warn=True)
        return (dpos, dchi, deta, st) if with_status else (dpos, dchi, deta)


class NotConvergedError(PQError):
    """A QEQ solve inside an autograd function stopped at max_it above its
    tolerance: the energy, the charges and the gradients (which hold only at
    the solution) would be wrong, so they are not returned."""

    def __init__(self, what, iterations, rel_residual, tol):
        RuntimeError.__init__(self, f"PQ_WARN_NOT_CONVERGED: {what} stopped after {iterations} products at relative "
                                    f"residual {rel_residual:.3e} > tol {tol:.1e}")
        self.code = PQ_WARN_NOT_CONVERGED
        self.iterations, self.rel_residual = iterations, rel_residual


def _solve_or_raise(context, chi, eta, q_tot, tol, max_it, restart, energy):
    r = context.qeq_solve(chi.detach(), eta.detach(), q_tot=q_tot, tol=tol, max_it=max_it, restart=restart,
                          energy=energy)
    if r.status != PQ_OK:
        raise NotConvergedError("QEQ solve", r.iterations, r.rel_residual, tol)
    return r


class QEQEnergy(torch.autograd.Function):
    """E(R, chi, u) = min_q E(R, q) on sum q = q_tot, with the hand-written
    adjoint (envelope theorem) as backward: dE/dR = -F[q*], dE/dchi = q*,
    dE/du = q*^2/2. The context must hold the system at positions `pos`.
    Raises NotConvergedError if the solve does not reach tol within max_it
    products (the envelope gradients hold only at the solution)."""

    @staticmethod
    def forward(ctx, pos, chi, eta, context: Context, q_tot: float = 0.0, tol: float = 1e-8, max_it: int = 500,
                restart: int = 50):
        r = _solve_or_raise(context, chi, eta, q_tot, tol, max_it, restart, True)
        ctx.context = context
        ctx.save_for_backward(chi.detach(), eta.detach(), r.q)
        return r.energy[0].clone()

    @staticmethod
    def backward(ctx, g):
        chi, eta, q = ctx.saved_tensors
        dpos, dchi, deta, _ = ctx.context.qeq_vjp(chi, eta, q, None, with_status=True)
        return g * dpos, g * dchi, g * deta, None, None, None, None, None


class QEQCharges(torch.autograd.Function):
    """q*(R, chi, u); backward solves the adjoint bordered system. Raises
    NotConvergedError if the solve or the adjoint solve does not reach tol
    within max_it products."""

    @staticmethod
    def forward(ctx, pos, chi, eta, context: Context, q_tot: float = 0.0, tol: float = 1e-8, max_it: int = 500,
                restart: int = 50):
        r = _solve_or_raise(context, chi, eta, q_tot, tol, max_it, restart, False)
        ctx.context, ctx.tol, ctx.max_it = context, tol, max_it
        ctx.save_for_backward(chi.detach(), eta.detach(), r.q)
        return r.q.clone()

    @staticmethod
    def backward(ctx, g):
        chi, eta, q = ctx.saved_tensors
        dpos, dchi, deta, st = ctx.context.qeq_vjp(chi, eta, q, g.contiguous(), tol=ctx.tol, max_it=ctx.max_it,
                                                   with_status=True)
        if st != PQ_OK:
            raise NotConvergedError("adjoint solve", -1, float("nan"), ctx.tol)
        return dpos, dchi, deta, None, None, None, None, None


def request_footprint(n: int, params: Params, restart: int = 50) -> float:
    """Device bytes that server admission charges for such a request."""
    v = load().pq_request_footprint(int(n), ctypes.byref(params), int(restart))
    if v < 0:
        raise ValueError("invalid request")
    return float(v)


class Server:
    """Continuous-batching QEQ server (host arrays in, host charges out)."""

    def __init__(self, device=0, slots=8, hbm_budget_bytes=64e9):
        self.lib = load()
        cfg = ServerCfg(device, slots, float(hbm_budget_bytes))
        h = ctypes.c_void_p()
        _check(self.lib.pq_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self.h = h
        self._keep = {}

    def submit(self, pos, chi, eta, params: Params, q0=None, q_tot=0.0, tol=1e-5, max_it=200, restart=50,
               solver="gmres") -> int:
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (pos, chi, eta)]
        q0a = None if q0 is None else np.ascontiguousarray(q0, dtype=np.float64)
        n = arrs[1].shape[0]
        req = Request(n, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                      None if q0a is None else q0a.ctypes.data, float(q_tot), float(tol), int(max_it), int(restart),
                      SOLVERS[solver], 0, params)
        t = ctypes.c_uint64()
        _check(self.lib.pq_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = n
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        import numpy as np
        n = self._keep[ticket]
        q = np.empty(n, dtype=np.float64)
        res = Result()
        res.q = q.ctypes.data
        code = self.lib.pq_server_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(res), int(timeout_us))
        if code == -9:
            return None
        _check(code)
        del self._keep[ticket]
        return dict(q=q, energy=res.energy, iterations=res.info.iterations, rel_residual=res.info.rel_residual,
                    status=res.status, t_submit=res.t_submit_s, t_start=res.t_start_s, t_done=res.t_done_s,
                    message=res.message.decode(errors="replace"))

    def close(self):
        if getattr(self, "h", None):
            _check(self.lib.pq_server_destroy(self.h))
            self.h = None
