"""FP64 CPU oracle of the hybrid LB/FD step (arXiv:1406.2686, Sec. 2).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``.  The product library never imports, loads or calls
anything here, and nothing here imports the product package.

``lbfd_oracle.c`` holds the stepping algorithm (stages S1-S11 in the paper's order);
this module is ctypes marshalling plus the paper's closed forms used as pins
(``tests/paper_closed_forms.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbfd_oracle.c")
_LIB = os.path.join(_HERE, "liblbfd_oracle.so")

PHASE = {"none": 0, "A": 1, "B": 2, "all": 3}
COUPLING = {"force": 0, "stress": 1}
COLLISION = {"bgk": 0, "mrt": 1}
FENE = {"upwind_euler": 0, "cholesky_ab2": 1}
FLAG_NONFINITE, FLAG_EXTENSIBILITY, FLAG_NOT_SPD = 1, 2, 4

DIAG_FIELDS = (
    "mass_A", "mass_B", "mom_x", "mom_y", "mom_z", "W", "xc", "yc", "zc",
    "Mxx", "Myy", "Mzz", "Mxy", "Mxz", "Myz", "D", "theta_deg",
    "min_L2_minus_trC", "min_minor", "max_u", "flags", "poly_trace_excess",
)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP over z-planes)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.c_int] * 4
        L.orc_destroy.argtypes = [P]
        L.orc_set_params.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_set_walls.argtypes = [P, D, D]
        L.orc_set_fields.argtypes = [P, D, D, D]
        L.orc_set_fields.restype = ctypes.c_int
        L.orc_step.argtypes = [P, ctypes.c_long]
        L.orc_step.restype = ctypes.c_int
        L.orc_steps.argtypes = [P]
        L.orc_steps.restype = ctypes.c_long
        L.orc_get_fields.argtypes = [P, D, D, D]
        L.orc_get_forces.argtypes = [P, D, D, D]
        L.orc_get_pops.argtypes = [P, D]
        L.orc_diagnostics.argtypes = [P, D]
        L.orc_lattice.argtypes = [I, D, I]
        L.orc_equilibrium.argtypes = [ctypes.c_double, D, D]
        L.orc_equilibrium_stress.argtypes = [ctypes.c_double, D, D, D]
        L.orc_source.argtypes = [D, D, D]
        L.orc_collide_node.argtypes = [D, ctypes.c_double, D, D, ctypes.c_double, D]
        L.orc_collide_node_mrt.argtypes = [D, ctypes.c_double, D, D, ctypes.c_double, D]
        L.orc_mrt_basis.argtypes = [D]
        L.orc_set_collision.argtypes = [P, ctypes.c_int]
        L.orc_set_fene.argtypes = [P, ctypes.c_int, ctypes.c_double]
        L.orc_cholesky_ab2.argtypes = [ctypes.c_double, D, D, D, ctypes.c_int, D, D,
                                       ctypes.POINTER(ctypes.c_int)]
        L.orc_fenep_kinematic.argtypes = [P, D, ctypes.c_long]
        L.orc_fenep_kinematic.restype = ctypes.c_int
        L.orc_get_C.argtypes = [P, D]
        L.orc_set_C.argtypes = [P, D]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (its results do not depend on it)."""
    lib().orc_set_threads(int(n))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _opt(a):
    return None if a is None else _dp(a)


def lattice():
    """D3Q19 velocities (19, 3), weights (19,), opposite map (19,)."""
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().orc_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                      opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c.reshape(19, 3), w, opp


def equilibrium(rho: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    E = np.zeros(19)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(E))
    return E



def equilibrium_stress(rho: float, u, Ts) -> np.ndarray:
    """Equilibrium whose second moment is lowered by the symmetric tensor Ts (xx, yy, zz,
    xy, xz, yz): the stress coupling of Sec. 2, eq. MODEtransformation."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    Ts = np.ascontiguousarray(Ts, dtype=np.float64)
    E = np.zeros(19)
    lib().orc_equilibrium_stress(float(rho), _dp(u), _dp(Ts), _dp(E))
    return E

def source(u, F) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    S = np.zeros(19)
    lib().orc_source(_dp(u), _dp(F), _dp(S))
    return S


def collide_node(f, rho, u, F, tau, collision="bgk") -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    fn = lib().orc_collide_node_mrt if collision == "mrt" else lib().orc_collide_node
    fn(_dp(f), float(rho), _dp(u), _dp(F), float(tau), _dp(out))
    return out


def cholesky_ab2(L2, C, RC, yprev=None):
    """One step of the Cholesky scheme at a node: C, dC/dt (6 each) and the previous rate of
    (ln l11, l21, ln l22, l31, l32, ln l33) (None: forward Euler).  Returns (C_new, rate, flag)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    RC = np.ascontiguousarray(RC, dtype=np.float64)
    yp = np.zeros(6) if yprev is None else np.ascontiguousarray(yprev, dtype=np.float64)
    cn, yd = np.zeros(6), np.zeros(6)
    flag = ctypes.c_int(0)
    lib().orc_cholesky_ab2(float(L2), _dp(C), _dp(RC), _dp(yp), 0 if yprev is None else 1, _dp(cn), _dp(yd),
                           ctypes.byref(flag))
    return cn, yd, int(flag.value)


def mrt_basis() -> np.ndarray:
    """The 19 x 19 moment basis of the MRT collision (rows: moments, columns: directions)."""
    M = np.zeros(19 * 19)
    lib().orc_mrt_basis(_dp(M))
    return M.reshape(19, 19)


class Oracle:
    """One lattice instance of the FP64 oracle.

    Grid axes: x and z periodic, y bounded by two moving walls (half-way, at y = -1/2
    and y = ny - 1/2).  Host field layout is SoA ``[field][z][y][x]`` flattened.
    """

    def __init__(self, nx: int, ny: int, nz: int, ncomp: int):
        self.nx, self.ny, self.nz, self.ncomp = nx, ny, nz, ncomp
        self.N = nx * ny * nz
        self._h = lib().orc_create(nx, ny, nz, ncomp)
        if not self._h:
            raise ValueError("oracle: invalid grid")

    def __del__(self):
        h = getattr(self, "_h", None)
        # at interpreter exit the module's globals may already be gone: the process is
        # ending and takes the oracle's memory with it
        if h and lib is not None:
            lib().orc_destroy(h)
            self._h = None

    def set_params(self, tau_A=1.0, tau_B=1.0, G=0.0, delta=0.1, polymer_phase="none",
                   eta_p=0.0, tau_p=1000.0, L2=100.0, coupling="force", collision="bgk",
                   fene="upwind_euler", kappa=0.0):
        ph = PHASE[polymer_phase] if isinstance(polymer_phase, str) else int(polymer_phase)
        cp = COUPLING[coupling] if isinstance(coupling, str) else int(coupling)
        lib().orc_set_params(self._h, tau_A, tau_B, G, delta, ph, eta_p, tau_p, L2, cp)
        lib().orc_set_collision(self._h, COLLISION[collision] if isinstance(collision, str) else int(collision))
        lib().orc_set_fene(self._h, FENE[fene] if isinstance(fene, str) else int(fene), float(kappa))

    def set_walls(self, u_bottom, u_top):
        ub = np.ascontiguousarray(u_bottom, dtype=np.float64)
        ut = np.ascontiguousarray(u_top, dtype=np.float64)
        lib().orc_set_walls(self._h, _dp(ub), _dp(ut))

    def set_fields(self, rho, u, C):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ncomp, self.N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, self.N)
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(6, self.N)
        lib().orc_set_fields(self._h, _dp(rho), _dp(u), _dp(C))

    def step(self, nsteps: int) -> int:
        return lib().orc_step(self._h, int(nsteps))

    @property
    def steps(self) -> int:
        return lib().orc_steps(self._h)

    def get_fields(self):
        rho = np.zeros((self.ncomp, self.N))
        u = np.zeros((3, self.N))
        C = np.zeros((6, self.N))
        lib().orc_get_fields(self._h, _dp(rho), _dp(u), _dp(C))
        return rho, u, C

    def get_forces(self):
        g = np.zeros((self.ncomp, 3, self.N))
        Fp = np.zeros((3, self.N))
        F = np.zeros((self.ncomp, 3, self.N))
        lib().orc_get_forces(self._h, _dp(g), _dp(Fp), _dp(F))
        return g, Fp, F

    def get_pops(self):
        f = np.zeros((self.ncomp, 19, self.N))
        lib().orc_get_pops(self._h, _dp(f))
        return f

    def diagnostics(self) -> dict:
        out = np.zeros(22)
        lib().orc_diagnostics(self._h, _dp(out))
        return dict(zip(DIAG_FIELDS, out.tolist()))

    def fenep_kinematic(self, u, nsteps: int) -> int:
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, self.N)
        return lib().orc_fenep_kinematic(self._h, _dp(u), int(nsteps))

    def get_C(self):
        C = np.zeros((6, self.N))
        lib().orc_get_C(self._h, _dp(C))
        return C

    def set_C(self, C):
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(6, self.N)
        lib().orc_set_C(self._h, _dp(C))


def from_workload(wl) -> Oracle:
    """Build an oracle instance from a workload dict produced by ``workloads``."""
    g = wl["grid"]
    o = Oracle(g["nx"], g["ny"], g["nz"], g["ncomp"])
    p = wl["params"]
    o.set_params(tau_A=p["tau_A"], tau_B=p["tau_B"], G=p["G"], delta=p["delta"],
                 polymer_phase=p["polymer_phase"], eta_p=p["eta_p"], tau_p=p["tau_p"],
                 L2=p["L2"], coupling=p.get("coupling", "force"), collision=p.get("collision", "bgk"),
                 fene=p.get("fene", "upwind_euler"), kappa=p.get("kappa", 0.0))
    o.set_walls(wl["walls"]["u_bottom"], wl["walls"]["u_top"])
    o.set_fields(wl["rho"], wl["u"], wl["C"])
    return o
