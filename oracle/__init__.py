"""ctypes wrapper of the CPU FP64 oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library
and the library never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_SRC = os.path.join(_HERE, "chorus_oracle.c")


def build(force=True):
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if (not force and os.path.exists(_LIB_PATH)
            and os.path.getmtime(_LIB_PATH) >= max(os.path.getmtime(_SRC),
                                                   os.path.getmtime(_SRC[:-1] + "h"))):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_basis.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        L.ora_basis.restype = ctypes.c_int
        L.ora_mesh_new.argtypes = [ctypes.c_int, ctypes.c_long, dp, ctypes.c_long,
                                   ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_long)]
        L.ora_mesh_new.restype = P
        L.ora_mesh_free.argtypes = [P]
        L.ora_error.restype = ctypes.c_char_p
        L.ora_solpts.argtypes = [P, dp, dp]
        L.ora_geometry.argtypes = [P, dp, dp, dp]
        L.ora_faces.argtypes = [P, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
        L.ora_residual.argtypes = [P, P, dp, dp]
        L.ora_residual_sgs.argtypes = [P, P, dp, dp, dp]
        L.ora_gradients.argtypes = [P, P, dp, dp]
        L.ora_rk3.argtypes = [P, P, dp, ctypes.c_double, ctypes.c_int]
        L.ora_ssp54.argtypes = [P, P, dp, ctypes.c_double, ctypes.c_int]
        L.ora_ssp54_table.argtypes = [dp, dp]
        L.ora_sums.argtypes = [P, dp, dp]
        L.ora_angular_momentum.argtypes = [P, dp, dp]
        L.ora_am_correct.argtypes = [P, dp, dp]
        L.ora_polytrope.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp, ctypes.c_double, dp, dp]
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP threads of the oracle's element loops (its results do not
    depend on the count)."""
    lib().omp_set_num_threads(int(n))


def max_threads():
    return int(lib().omp_get_max_threads())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OraPhys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("R_gas", ctypes.c_double), ("GM", ctypes.c_double),
                ("omega", ctypes.c_double), ("nu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("kappa_r", ctypes.c_double), ("T_top", ctypes.c_double),
                ("F_bottom", ctypes.c_double), ("bc_state", ctypes.c_double * 5),
                ("kappa_r1", ctypes.c_double), ("kappa_r2", ctypes.c_double)]


def phys(gamma=5.0 / 3.0, R_gas=1.0, GM=0.0, omega=0.0, nu=0.0, kappa=0.0, kappa_r=0.0,
         T_top=0.0, F_bottom=0.0, bc_state=(1.0, 0.0, 0.0, 0.0, 1.5), kappa_r1=0.0, kappa_r2=0.0):
    """Physics of the oracle; the radiative diffusivity at radius r is
    kappa_r + kappa_r1 r + kappa_r2 r^2."""
    p = OraPhys()
    p.gamma, p.R_gas, p.GM, p.omega = gamma, R_gas, GM, omega
    p.nu, p.kappa, p.kappa_r, p.T_top, p.F_bottom = nu, kappa, kappa_r, T_top, F_bottom
    p.kappa_r1, p.kappa_r2 = kappa_r1, kappa_r2
    for i in range(5):
        p.bc_state[i] = bc_state[i]
    return p


def ssp54_table():
    """(alpha, beta) [5][5] of the SSPRK(5,4) Shu-Osher form (row = stage)."""
    a = np.zeros(25)
    b = np.zeros(25)
    lib().ora_ssp54_table(_dp(a), _dp(b))
    return a.reshape(5, 5), b.reshape(5, 5)


def basis(N):
    """(xs, xf, I, D, w) of the 1D SD operators of order N."""
    xs = np.zeros(N)
    xf = np.zeros(N + 1)
    I = np.zeros((N + 1, N))
    D = np.zeros((N, N + 1))
    w = np.zeros(N)
    rc = lib().ora_basis(N, _dp(xs), _dp(xf), _dp(I), _dp(D), _dp(w))
    if rc != 0:
        raise ValueError("unsupported order %d" % N)
    return xs, xf, I, D, w


class OracleMesh:
    """Oracle geometry and operators on a hex20 mesh (chorus_inputs.Hex20Mesh)."""

    def __init__(self, mesh, N):
        L = lib()
        self.N = int(N)
        self.E = mesh.n_elems
        self.np = self.N ** 3
        self._xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        self._e20 = np.ascontiguousarray(mesh.elem20, dtype=np.int64)
        self._bc = np.ascontiguousarray(mesh.face_bc, dtype=np.int32)
        self._mid = np.ascontiguousarray(mesh.match_id, dtype=np.int64)
        h = L.ora_mesh_new(self.N, mesh.n_nodes, _dp(self._xyz), self.E,
                           self._e20.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                           self._bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           self._mid.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
        if not h:
            raise ValueError("oracle mesh: " + L.ora_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_mesh_free(h)
            self._h = None

    @property
    def n_solpts(self):
        return self.E * self.np

    def solpts(self):
        xyz = np.zeros((3, self.n_solpts))
        wJ = np.zeros(self.n_solpts)
        lib().ora_solpts(self._h, _dp(xyz), _dp(wJ))
        return xyz, wJ

    def geometry(self):
        N = self.N
        jac = np.zeros(self.n_solpts)
        met = np.zeros((self.n_solpts, 3, 3))
        metf = np.zeros((self.E, 3, (N + 1) * N * N, 3))
        lib().ora_geometry(self._h, _dp(jac), _dp(met), _dp(metf))
        return jac, met, metf

    def faces(self):
        ne = np.zeros(self.E * 6, dtype=np.int64)
        nf = np.zeros(self.E * 6, dtype=np.int32)
        npnt = np.zeros(self.E * 6 * self.N ** 2, dtype=np.int32)
        lib().ora_faces(self._h, ne.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                        nf.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        npnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return ne.reshape(self.E, 6), nf.reshape(self.E, 6), npnt.reshape(self.E, 6, self.N ** 2)

    def residual(self, ph, Q, sgs=None):
        """dQ/dt [5][E][N^3]; sgs: optional additional Cartesian flux
        [15][E][N^3] (v*3+c) at the solution points."""
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(5, self.E, self.np)
        R = np.zeros_like(Q)
        if sgs is None:
            lib().ora_residual(self._h, ctypes.byref(ph), _dp(Q), _dp(R))
        else:
            sg = np.ascontiguousarray(sgs, dtype=np.float64).reshape(15, self.E, self.np)
            lib().ora_residual_sgs(self._h, ctypes.byref(ph), _dp(Q), _dp(sg), _dp(R))
        return R

    def gradients(self, ph, Q):
        """BR1 gradients of the conserved variables [15][E][N^3] (v*3+c)."""
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(5, self.E, self.np)
        G = np.zeros((15, self.E, self.np))
        lib().ora_gradients(self._h, ctypes.byref(ph), _dp(Q), _dp(G))
        return G

    def rk3(self, ph, Q, dt, nsteps):
        Q = np.array(Q, dtype=np.float64, order="C", copy=True).reshape(5, self.E, self.np)
        lib().ora_rk3(self._h, ctypes.byref(ph), _dp(Q), float(dt), int(nsteps))
        return Q

    def ssp54(self, ph, Q, dt, nsteps):
        """nsteps of the five-stage fourth-order SSP Runge-Kutta method."""
        Q = np.array(Q, dtype=np.float64, order="C", copy=True).reshape(5, self.E, self.np)
        lib().ora_ssp54(self._h, ctypes.byref(ph), _dp(Q), float(dt), int(nsteps))
        return Q

    def sums(self, Q):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        out = np.zeros(5)
        lib().ora_sums(self._h, _dp(Q), _dp(out))
        return out

    def angular_momentum(self, Q):
        """(L [3], I [3]) of the state (Section 6)."""
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        out = np.zeros(6)
        lib().ora_angular_momentum(self._h, _dp(Q), _dp(out))
        return out[:3], out[3:]

    def am_correct(self, Q):
        """(corrected copy of Q, applied dOmega [3])."""
        Q = np.array(Q, dtype=np.float64, order="C", copy=True)
        dO = np.zeros(3)
        lib().ora_am_correct(self._h, _dp(Q), _dp(dO))
        return Q, dO

    def polytrope(self, beta, n_rho, poly_n=1.5, gamma=5.0 / 3.0, R_gas=1.0, noise=None, amp=1e-4):
        Q = np.zeros((5, self.E, self.np))
        pars = np.zeros(4)
        nz = None
        if noise is not None:
            nz = np.ascontiguousarray(noise, dtype=np.float64).reshape(-1)
            assert nz.size == self.n_solpts
        lib().ora_polytrope(self._h, beta, n_rho, poly_n, gamma, R_gas,
                            _dp(nz) if nz is not None else None, amp, _dp(Q), _dp(pars))
        return Q, dict(chi_o=pars[0], c=pars[1], alpha=pars[2], GM=pars[3])
