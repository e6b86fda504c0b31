"""Python binding of liblbfd, the gfx950 library for the hybrid lattice-Boltzmann /
finite-difference step of arXiv:1406.2686 (Shan-Chen D3Q19 + FENE-P).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch supplies the device memory (one caller-owned buffer per lattice) and the HIP
stream.  If the compiled library is missing this module raises at import; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbfd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_1406_2686_amd/build.py` (hipcc, gfx950)")

# torch carries its own HIP runtime library; it is loaded first so that the library binds to
# that one (a second runtime loaded for the library would not see torch's device memory)
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EEXTENSIBILITY, ENOTSPD, ESTATE = range(8)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENONFINITE",
                5: "EEXTENSIBILITY", 6: "ENOTSPD", 7: "ESTATE"}
FLAG_NONFINITE, FLAG_EXTENSIBILITY, FLAG_NOT_SPD = 1, 2, 4
POLYMER = {"none": 0, "A": 1, "B": 2, "all": 3}
COUPLING = {"force": 0, "stress": 1}
COLLISION = {"bgk": 0, "mrt": 1}
FENE = {"upwind_euler": 0, "cholesky_ab2": 1}


class LbfdError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ncomp", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("tau_A", ctypes.c_double), ("tau_B", ctypes.c_double), ("G", ctypes.c_double),
                ("delta", ctypes.c_double), ("rho0", ctypes.c_double * 2),
                ("polymer_phase", ctypes.c_int32), ("coupling", ctypes.c_int32),
                ("eta_p", ctypes.c_double), ("tau_p", ctypes.c_double), ("L2", ctypes.c_double),
                ("collision", ctypes.c_int32), ("fene_scheme", ctypes.c_int32), ("fene_kappa", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double * 2), ("momentum", ctypes.c_double * 3),
                ("W", ctypes.c_double), ("centroid", ctypes.c_double * 3),
                ("M", ctypes.c_double * 6), ("D", ctypes.c_double), ("theta_deg", ctypes.c_double),
                ("min_L2_minus_trC", ctypes.c_double), ("min_minor", ctypes.c_double),
                ("max_u", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("step", ctypes.c_int64),
                ("poly_trace_excess", ctypes.c_double)]

    def to_dict(self):
        return {"mass_A": self.mass[0], "mass_B": self.mass[1], "mom_x": self.momentum[0],
                "mom_y": self.momentum[1], "mom_z": self.momentum[2], "W": self.W,
                "xc": self.centroid[0], "yc": self.centroid[1], "zc": self.centroid[2],
                "Mxx": self.M[0], "Myy": self.M[1], "Mzz": self.M[2], "Mxy": self.M[3],
                "Mxz": self.M[4], "Myz": self.M[5], "D": self.D, "theta_deg": self.theta_deg,
                "min_L2_minus_trC": self.min_L2_minus_trC, "min_minor": self.min_minor,
                "max_u": self.max_u, "flags": int(self.flags), "step": int(self.step),
                "poly_trace_excess": self.poly_trace_excess}


class Walls(ctypes.Structure):
    _fields_ = [("u_bottom", ctypes.c_double * 3), ("u_top", ctypes.c_double * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("tile", ctypes.c_int32), ("zchunk", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


PATH_FUSED, PATH_SPLIT, PATH_TWOPASS, PATH_CHAINED = 0, 1, 2, 3
TILES = {"32x8": 0, "32x16": 1, "16x16": 2, "64x8": 3}

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


def _sig(name, args, res=ctypes.c_int32):
    fn = getattr(_lib, name)
    fn.argtypes = args
    fn.restype = res
    return fn


_sig("lbfd_state_bytes", [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_uint64)])
_sig("lbfd_create", [ctypes.POINTER(Grid), ctypes.POINTER(Params), _P, ctypes.c_uint64, _P,
                     ctypes.POINTER(_P)])
_sig("lbfd_set_params", [_P, ctypes.POINTER(Params)])
_sig("lbfd_set_walls", [_P, _D, _D])
_sig("lbfd_set_fields", [_P, _D, _D, _D])
_sig("lbfd_set_fields_box", [_P, _I32, _I32, _I32, _I32, _I32, _I32, _D, _D, _D])
_sig("lbfd_reset_counters", [_P])
_sig("lbfd_step", [_P, _I64])
_sig("lbfd_step_async", [_P, _I64])
_sig("lbfd_get_flags", [_P, ctypes.POINTER(ctypes.c_uint32)])
_sig("lbfd_fenep_kinematic", [_P, _D, _I64])
_sig("lbfd_get_fields", [_P, _D, _D, _D])
_sig("lbfd_get_fields_box", [_P, _I32, _I32, _I32, _I32, _I32, _I32, _D, _D, _D])
_sig("lbfd_diagnostics", [_P, ctypes.POINTER(Diag)])
_sig("lbfd_diagnostics_noalloc", [_P, ctypes.POINTER(Diag)])
_sig("lbfd_checkpoint_bytes", [_P, ctypes.POINTER(ctypes.c_uint64)])
_sig("lbfd_get_state", [_P, _P, ctypes.c_uint64])
_sig("lbfd_set_state", [_P, _P, ctypes.c_uint64])
_sig("lbfd_set_tuning", [_P, ctypes.POINTER(Tuning)])
_sig("lbfd_get_tuning", [_P, ctypes.POINTER(Tuning)])
class SteadyCrit(ctypes.Structure):
    _fields_ = [("every", ctypes.c_int32), ("window", ctypes.c_int32), ("tol", ctypes.c_double),
                ("windows", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_sig("lbfd_autotune", [_P, ctypes.c_int32, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)])
_sig("lbfd_batch_state_bytes", [ctypes.c_int32, ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_uint64)])
_sig("lbfd_batch_create", [ctypes.c_int32, ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.POINTER(Walls), _P,
                           ctypes.c_uint64, _P, ctypes.POINTER(_P)])
_sig("lbfd_batch_set_fields", [_P, ctypes.c_int32, _D, _D, _D])
_sig("lbfd_batch_set_tuning", [_P, ctypes.POINTER(Tuning)])
_sig("lbfd_batch_get_tuning", [_P, ctypes.POINTER(Tuning)])
_sig("lbfd_batch_set_active", [_P, ctypes.POINTER(ctypes.c_uint8)])
_sig("lbfd_batch_step", [_P, _I64])
_sig("lbfd_batch_diagnostics", [_P, ctypes.POINTER(Diag)])
_sig("lbfd_batch_get_fields", [_P, ctypes.c_int32, _D, _D, _D])
_sig("lbfd_batch_run_to_steady", [_P, ctypes.POINTER(SteadyCrit), _I64, ctypes.POINTER(Diag),
                                  ctypes.POINTER(ctypes.c_int64)])
_sig("lbfd_batch_autotune", [_P, ctypes.c_int32, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)])
PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p)
_sig("lbfd_batch_set_progress", [_P, PROGRESS_FN, _P])
_sig("lbfd_batch_instance", [_P, ctypes.c_int32], _P)
_sig("lbfd_batch_destroy", [_P], None)
_sig("lbfd_batch_last_error", [_P], ctypes.c_char_p)
class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


_F = ctypes.POINTER(ctypes.c_float)
_sig("lbfd_mlp_state_bytes", [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)])
_sig("lbfd_mlp_create", [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _P, ctypes.c_uint64, _P,
                         ctypes.POINTER(_P)])
_sig("lbfd_mlp_set_params", [_P, _F])
_sig("lbfd_mlp_get_params", [_P, _F])
_sig("lbfd_mlp_forward", [_P, _F, ctypes.c_int32, _F])
_sig("lbfd_mlp_loss_grad", [_P, _F, _F, ctypes.c_int32, _F, _F])
_sig("lbfd_mlp_adam_step", [_P, ctypes.POINTER(TrainOpts)])
_sig("lbfd_mlp_train", [_P, _F, _F, ctypes.c_int32, ctypes.POINTER(TrainOpts), _F])
_sig("lbfd_mlp_infer_bf16", [_P, _F, ctypes.c_int32, _F])
_sig("lbfd_mlp_destroy", [_P], None)
_sig("lbfd_mlp_last_error", [_P], ctypes.c_char_p)
_sig("lbfd_version", [], ctypes.c_char_p)
_sig("lbfd_stream_probe", [ctypes.c_int32, _P, _P, ctypes.c_uint64, ctypes.c_int32, _P,
                           ctypes.POINTER(ctypes.c_double)])
PROBES = {"read": 0, "write": 1, "write_nt": 2, "copy": 3, "copy_nt": 4}


def stream_probe(kind: str, nbytes: int, reps: int = 20, device="cuda") -> dict:
    """HBM streaming rate of the library's probe kernel `kind` (read, write, write_nt, copy,
    copy_nt) over buffers of nbytes each: ms per launch and GB/s of bytes moved."""
    import torch

    nbytes = nbytes // 16 * 16
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    ms = ctypes.c_double(0)
    stream = torch.cuda.current_stream(src.device)
    st = _lib.lbfd_stream_probe(PROBES[kind], _P(src.data_ptr()), _P(dst.data_ptr()), ctypes.c_uint64(nbytes),
                                int(reps), _P(stream.cuda_stream), ctypes.byref(ms))
    if st != OK:
        raise LbfdError(st, "lbfd_stream_probe")
    moved = nbytes * (2 if kind.startswith("copy") else 1)
    return {"kind": kind, "bytes": moved, "ms": ms.value, "GB_per_s": moved / (ms.value * 1e-3) / 1e9}
_sig("lbfd_destroy", [_P], None)
_sig("lbfd_last_error", [_P], ctypes.c_char_p)


def raw():
    """The ctypes handle of liblbfd (for ABI-level tests)."""
    return _lib


def version() -> str:
    return _lib.lbfd_version().decode()


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def make_params(tau_A=1.0, tau_B=1.0, G=0.0, delta=0.1, rho0=(1.0, 0.0), polymer_phase="none",
                eta_p=0.0, tau_p=1000.0, L2=100.0, coupling="force", collision="bgk", fene="upwind_euler",
                kappa=0.0, **_ignored) -> Params:
    ph = POLYMER[polymer_phase] if isinstance(polymer_phase, str) else int(polymer_phase)
    cp = COUPLING[coupling] if isinstance(coupling, str) else int(coupling)
    co = COLLISION[collision] if isinstance(collision, str) else int(collision)
    fs = FENE[fene] if isinstance(fene, str) else int(fene)
    r0 = list(rho0) + [0.0] * (2 - len(rho0))
    return Params(float(tau_A), float(tau_B), float(G), float(delta),
                  (ctypes.c_double * 2)(*r0), ph, cp, float(eta_p), float(tau_p), float(L2), co, fs,
                  float(kappa))


def state_bytes(nx, ny, nz, ncomp) -> int:
    g = Grid(nx, ny, nz, ncomp)
    b = ctypes.c_uint64(0)
    st = _lib.lbfd_state_bytes(ctypes.byref(g), ctypes.byref(b))
    if st != OK:
        raise LbfdError(st, "invalid grid")
    return int(b.value)


class Lattice:
    """One lattice on the current GPU.  Device state lives in a torch uint8 tensor."""

    def __init__(self, nx, ny, nz, ncomp, params: Params | dict, device="cuda", stream=None):
        import torch

        self.nx, self.ny, self.nz, self.ncomp = int(nx), int(ny), int(nz), int(ncomp)
        self.N = self.nx * self.ny * self.nz
        self.grid = Grid(self.nx, self.ny, self.nz, self.ncomp)
        nbytes = state_bytes(self.nx, self.ny, self.nz, self.ncomp)
        self.device = torch.device(device)
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        p = params if isinstance(params, Params) else make_params(**params)
        h = _P()
        with torch.cuda.device(self.device):
            st = _lib.lbfd_create(ctypes.byref(self.grid), ctypes.byref(p), _P(aligned),
                                  ctypes.c_uint64(nbytes), _P(self._stream.cuda_stream),
                                  ctypes.byref(h))
        if st != OK:
            raise LbfdError(st, "lbfd_create failed")
        self._h = h

    # -- helpers
    def _check(self, st):
        if st != OK:
            raise LbfdError(st, _lib.lbfd_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbfd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return self._stream

    def set_params(self, params):
        p = params if isinstance(params, Params) else make_params(**params)
        self._check(_lib.lbfd_set_params(self._h, ctypes.byref(p)))

    def set_walls(self, u_bottom, u_top):
        ub = np.ascontiguousarray(u_bottom, dtype=np.float64)
        ut = np.ascontiguousarray(u_top, dtype=np.float64)
        self._check(_lib.lbfd_set_walls(self._h, _dp(ub), _dp(ut)))

    def set_fields(self, rho, u, C):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ncomp, self.N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, self.N)
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(6, self.N)
        self._check(_lib.lbfd_set_fields(self._h, _dp(rho), _dp(u), _dp(C)))

    def set_fields_box(self, x0, y0, z0, bx, by, bz, rho, u, C):
        B = bx * by * bz
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ncomp, B)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, B)
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(6, B)
        self._check(_lib.lbfd_set_fields_box(self._h, x0, y0, z0, bx, by, bz, _dp(rho), _dp(u),
                                             _dp(C)))

    def reset_counters(self):
        self._check(_lib.lbfd_reset_counters(self._h))

    def step(self, n: int):
        self._check(_lib.lbfd_step(self._h, int(n)))

    def step_status(self, n: int) -> int:
        """Like step() but returns the status code instead of raising."""
        return int(_lib.lbfd_step(self._h, int(n)))

    def step_async(self, n: int):
        self._check(_lib.lbfd_step_async(self._h, int(n)))

    def fenep_kinematic(self, u, n: int):
        """Advance C by n FENE-P steps under the prescribed velocity u (3, N), the
        lattice-Boltzmann part switched off (lbfd_fenep_kinematic)."""
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, self.N)
        self._check(_lib.lbfd_fenep_kinematic(self._h, _dp(u), int(n)))

    def flags(self) -> int:
        f = ctypes.c_uint32(0)
        self._check(_lib.lbfd_get_flags(self._h, ctypes.byref(f)))
        return int(f.value)

    def get_fields(self):
        rho = np.zeros((self.ncomp, self.N))
        u = np.zeros((3, self.N))
        C = np.zeros((6, self.N))
        self._check(_lib.lbfd_get_fields(self._h, _dp(rho), _dp(u), _dp(C)))
        return rho, u, C

    def get_fields_box(self, x0, y0, z0, bx, by, bz):
        B = bx * by * bz
        rho = np.zeros((self.ncomp, B))
        u = np.zeros((3, B))
        C = np.zeros((6, B))
        self._check(_lib.lbfd_get_fields_box(self._h, x0, y0, z0, bx, by, bz, _dp(rho), _dp(u),
                                             _dp(C)))
        return rho, u, C

    def set_tuning(self, path=PATH_FUSED, tile="32x8", zchunk=0):
        t = Tuning(int(path), TILES[tile] if isinstance(tile, str) else int(tile), int(zchunk), 0)
        self._check(_lib.lbfd_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(_lib.lbfd_get_tuning(self._h, ctypes.byref(t)))
        inv = {v: k for k, v in TILES.items()}
        return {"path": int(t.path), "tile": inv[int(t.tile)], "zchunk": int(t.zchunk)}

    def autotune(self, reps: int = 3) -> dict:
        """Time every launch shape that implements the lattice's options on the current
        state (which is left unchanged) and keep the fastest; returns the chosen shape and
        its ms per step."""
        t = Tuning()
        ms = ctypes.c_double(0)
        self._check(_lib.lbfd_autotune(self._h, int(reps), ctypes.byref(t), ctypes.byref(ms)))
        inv = {v: k for k, v in TILES.items()}
        return {"path": int(t.path), "tile": inv[int(t.tile)], "zchunk": int(t.zchunk),
                "ms_per_step": float(ms.value)}

    def diagnostics(self) -> dict:
        d = Diag()
        self._check(_lib.lbfd_diagnostics(self._h, ctypes.byref(d)))
        return d.to_dict()

    def diagnostics_noalloc(self) -> dict:
        """The record of diagnostics(), reduced through the library's static per-device
        scratch instead of the lattice's buffer (lbfd_diagnostics_noalloc)."""
        d = Diag()
        self._check(_lib.lbfd_diagnostics_noalloc(self._h, ctypes.byref(d)))
        return d.to_dict()

    def get_state(self) -> bytes:
        n = ctypes.c_uint64(0)
        self._check(_lib.lbfd_checkpoint_bytes(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(_lib.lbfd_get_state(self._h, ctypes.cast(buf, _P), n))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(_lib.lbfd_set_state(self._h, ctypes.cast(buf, _P), ctypes.c_uint64(len(blob))))


def from_workload(wl, device="cuda") -> Lattice:
    """Create a lattice from a workload dict (see workloads.py) and upload its fields."""
    g = wl["grid"]
    lat = Lattice(g["nx"], g["ny"], g["nz"], g["ncomp"], wl["params"], device=device)
    lat.set_walls(wl["walls"]["u_bottom"], wl["walls"]["u_top"])
    lat.set_fields(wl["rho"], wl["u"], wl["C"])
    return lat


class Batch:
    """n independent lattices (same ncomp) stepped by one launch per step.  A dedicated
    non-default torch stream is used so that the step graph can be captured."""

    def __init__(self, workloads_list, device="cuda"):
        import torch

        self.n = len(workloads_list)
        self.device = torch.device(device)
        grids = (Grid * self.n)(*[Grid(w["grid"]["nx"], w["grid"]["ny"], w["grid"]["nz"],
                                       w["grid"]["ncomp"]) for w in workloads_list])
        params = (Params * self.n)(*[make_params(**w["params"]) for w in workloads_list])
        walls = (Walls * self.n)(*[Walls((ctypes.c_double * 3)(*w["walls"]["u_bottom"]),
                                         (ctypes.c_double * 3)(*w["walls"]["u_top"])) for w in workloads_list])
        nb = ctypes.c_uint64(0)
        st = _lib.lbfd_batch_state_bytes(self.n, grids, ctypes.byref(nb))
        if st != OK:
            raise LbfdError(st, "invalid batch grids")
        self._buf = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._buf.data_ptr() + 255) // 256 * 256
        self._stream = torch.cuda.Stream(device=self.device)
        h = _P()
        with torch.cuda.device(self.device):
            st = _lib.lbfd_batch_create(self.n, grids, params, walls, _P(aligned), nb,
                                        _P(self._stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise LbfdError(st, "lbfd_batch_create failed")
        self._h = h
        self.grids = [(g.nx, g.ny, g.nz, g.ncomp) for g in grids]
        for i, w in enumerate(workloads_list):
            self.set_fields(i, w["rho"], w["u"], w["C"])

    def _check(self, st):
        if st != OK:
            raise LbfdError(st, _lib.lbfd_batch_last_error(self._h).decode())

    @property
    def stream(self):
        return self._stream

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbfd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, i, rho, u, C):
        nx, ny, nz, nc = self.grids[i]
        N = nx * ny * nz
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(nc, N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, N)
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(6, N)
        self._check(_lib.lbfd_batch_set_fields(self._h, i, _dp(rho), _dp(u), _dp(C)))

    def set_tuning(self, tile="32x8", zchunk=0, path=PATH_FUSED):
        """Launch shape of the batched step: the fused body (tiles 32x8, 16x16) or the
        chained body (path=PATH_CHAINED, tiles 64x8 or 32x16)."""
        t = Tuning(int(path), TILES[tile] if isinstance(tile, str) else int(tile), int(zchunk), 0)
        self._check(_lib.lbfd_batch_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(_lib.lbfd_batch_get_tuning(self._h, ctypes.byref(t)))
        inv = {v: k for k, v in TILES.items()}
        return {"path": int(t.path), "tile": inv[int(t.tile)], "zchunk": int(t.zchunk)}

    def autotune(self, reps: int = 3) -> dict:
        t = Tuning()
        ms = ctypes.c_double(0)
        self._check(_lib.lbfd_batch_autotune(self._h, int(reps), ctypes.byref(t), ctypes.byref(ms)))
        inv = {v: k for k, v in TILES.items()}
        return {"path": int(t.path), "tile": inv[int(t.tile)], "zchunk": int(t.zchunk),
                "ms_per_step": float(ms.value)}

    def set_active(self, active):
        a = (ctypes.c_uint8 * self.n)(*[1 if x else 0 for x in active])
        self._check(_lib.lbfd_batch_set_active(self._h, a))

    def step(self, n: int):
        self._check(_lib.lbfd_batch_step(self._h, int(n)))

    def diagnostics(self):
        d = (Diag * self.n)()
        self._check(_lib.lbfd_batch_diagnostics(self._h, d))
        return [x.to_dict() for x in d]

    def get_fields(self, i):
        nx, ny, nz, nc = self.grids[i]
        N = nx * ny * nz
        rho = np.zeros((nc, N))
        u = np.zeros((3, N))
        C = np.zeros((6, N))
        self._check(_lib.lbfd_batch_get_fields(self._h, i, _dp(rho), _dp(u), _dp(C)))
        return rho, u, C

    def run_to_steady(self, every=100, window=1000, tol=1e-4, max_steps=100000, windows=1, progress=None):
        """Step until each instance's D moved less than tol over each of the last `windows`
        windows (or max_steps); returns final diagnostics and the steady step per instance
        (-1 not steady, -2 fault).  progress: optional callable(step, active) called after
        each `every` steps."""
        crit = SteadyCrit(int(every), int(window), float(tol), int(windows), 0)
        d = (Diag * self.n)()
        ss = (ctypes.c_int64 * self.n)()
        cb = PROGRESS_FN(lambda step, active, _user: progress(int(step), int(active))) if progress else PROGRESS_FN()
        self._check(_lib.lbfd_batch_set_progress(self._h, cb, None))
        try:
            self._check(_lib.lbfd_batch_run_to_steady(self._h, ctypes.byref(crit), int(max_steps), d, ss))
        finally:
            self._check(_lib.lbfd_batch_set_progress(self._h, PROGRESS_FN(), None))
        return [x.to_dict() for x in d], [int(v) for v in ss]


MLP_NPARAMS = 17667


def _fp(a):
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_F)


class MLP:
    """The 5 -> 128 -> 128 -> 3 GELU surrogate on the GPU (training FP32, inference BF16)."""

    def __init__(self, max_batch=512, max_train=4096, seed=0, device="cuda"):
        import torch

        nb = ctypes.c_uint64(0)
        st = _lib.lbfd_mlp_state_bytes(int(max_batch), int(max_train), ctypes.byref(nb))
        if st != OK:
            raise LbfdError(st, "lbfd_mlp_state_bytes")
        self.device = torch.device(device)
        self._buf = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._buf.data_ptr() + 255) // 256 * 256
        self._stream = torch.cuda.current_stream(self.device)
        h = _P()
        with torch.cuda.device(self.device):
            st = _lib.lbfd_mlp_create(int(max_batch), int(max_train), ctypes.c_uint64(seed), _P(aligned),
                                      nb, _P(self._stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise LbfdError(st, "lbfd_mlp_create")
        self._h = h
        self.max_batch = int(max_batch)

    def _check(self, st):
        if st != OK:
            raise LbfdError(st, _lib.lbfd_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbfd_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == MLP_NPARAMS
        self._check(_lib.lbfd_mlp_set_params(self._h, _fp(p)))

    def get_params(self):
        p = np.zeros(MLP_NPARAMS, dtype=np.float32)
        self._check(_lib.lbfd_mlp_get_params(self._h, _fp(p)))
        return p

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros((X.shape[0], 3), dtype=np.float32)
        self._check(_lib.lbfd_mlp_forward(self._h, _fp(X), X.shape[0], _fp(Y)))
        return Y

    def infer_bf16(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros((X.shape[0], 3), dtype=np.float32)
        self._check(_lib.lbfd_mlp_infer_bf16(self._h, _fp(X), X.shape[0], _fp(Y)))
        return Y

    def loss_grad(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        g = np.zeros(MLP_NPARAMS, dtype=np.float32)
        self._check(_lib.lbfd_mlp_loss_grad(self._h, _fp(X), _fp(T), X.shape[0], _fp(loss), _fp(g)))
        return float(loss[0]), g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        o = TrainOpts(1, 1, lr, beta1, beta2, eps, 0)
        self._check(_lib.lbfd_mlp_adam_step(self._h, ctypes.byref(o)))

    def train(self, X, T, epochs=200, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        o = TrainOpts(int(epochs), int(batch), lr, beta1, beta2, eps, int(seed))
        loss = np.zeros(1, dtype=np.float32)
        self._check(_lib.lbfd_mlp_train(self._h, _fp(X), _fp(T), X.shape[0], ctypes.byref(o), _fp(loss)))
        return float(loss[0])
