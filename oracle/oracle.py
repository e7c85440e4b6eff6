"""ctypes wrapper around the CPU FP64 oracle (oracle/liborc.so).

TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The functions mirror the oracle's C entry
points; every array is a plain numpy array on the host.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

BLOCK_CH = 0
BLOCK_NS = 1

PHI0_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_double), C.c_void_p)


class Params(C.Structure):
    """Non-dimensional parameters (Sec. 2): Cn, Pe, Re, We, Fr, the density and
    viscosity ratios rho_-/rho_+ and eta_-/eta_+, the time step, the unit
    gravity direction, C_I of tau_m and the mass-flux reading."""
    _fields_ = [("Cn", C.c_double), ("Pe", C.c_double), ("Re", C.c_double),
                ("We", C.c_double), ("Fr", C.c_double), ("rho_minus", C.c_double),
                ("eta_minus", C.c_double), ("dt", C.c_double), ("g", C.c_double * 3),
                ("C_I", C.c_double), ("flux_mode", C.c_int)]

    @classmethod
    def make(cls, Cn, Pe, Re, We, Fr, rho_minus, eta_minus, dt, g=(0.0, -1.0, 0.0),
             C_I=6.0, flux_mode=0):
        return cls(Cn, Pe, Re, We, Fr, rho_minus, eta_minus, dt, (C.c_double * 3)(*g),
                   C_I, flux_mode)


class SolverOpts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("newton_atol", C.c_double),
                ("block_tol", C.c_double), ("gmres_rtol", C.c_double),
                ("newton_max_it_ch", C.c_int), ("newton_max_it_ns", C.c_int),
                ("gmres_restart", C.c_int), ("gmres_max_it", C.c_int),
                ("block_max_it", C.c_int), ("block_min_it", C.c_int), ("precond", C.c_int)]

    @classmethod
    def make(cls, newton_rtol=1e-8, newton_atol=1e-12, block_tol=1e-4, gmres_rtol=1e-7,
             newton_max_it_ch=20, newton_max_it_ns=40, gmres_restart=30, gmres_max_it=1000,
             block_max_it=10, block_min_it=1, precond=1):
        return cls(newton_rtol, newton_atol, block_tol, gmres_rtol, newton_max_it_ch,
                   newton_max_it_ns, gmres_restart, gmres_max_it, block_max_it,
                   block_min_it, precond)


class StepStats(C.Structure):
    _fields_ = [("block_its", C.c_int), ("newton_its", C.c_int * 2), ("gmres_its", C.c_int * 2),
                ("converged", C.c_int), ("rel_res", C.c_double * 2), ("mass", C.c_double),
                ("energy", C.c_double)]


_lib = None


def build(verbose=False):
    from . import build_oracle
    return build_oracle.build(verbose)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_last_error.restype = C.c_char_p
        L.orc_mesh_build.argtypes = [C.POINTER(C.c_int32), C.c_int, C.c_int, PHI0_FN, C.c_void_p,
                                     C.c_double, C.POINTER(C.c_int32), C.c_int64,
                                     C.POINTER(C.c_void_p)]
        L.orc_mesh_free.argtypes = [C.c_void_p]
        L.orc_mesh_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_mesh_arrays.argtypes = [C.c_void_p] + [C.c_void_p] * 8
        L.orc_residual.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, dp, dp, dp, dp, dp]
        L.orc_jvp.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, dp, dp, dp, dp]
        L.orc_jvp_full.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, dp, dp, dp, dp]
        L.orc_residual_rows.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, dp, dp,
                                        C.POINTER(C.c_int32), C.c_int64, dp, dp]
        L.orc_diag_blocks.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int, dp, dp, dp]
        L.orc_diagnostics.argtypes = [C.c_void_p, C.POINTER(Params), dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.POINTER(Params), C.POINTER(SolverOpts), dp, dp, dp,
                               C.POINTER(StepStats)]
        L.orc_q2_build.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        L.orc_q2_free.argtypes = [C.c_void_p]
        L.orc_q2_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_q2_arrays.argtypes = [C.c_void_p] + [C.c_void_p] * 7
        L.orc_q2_residual.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(Params), C.c_int, dp, dp, dp]
        L.orc_q2_jvp.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(Params), C.c_int, dp, dp, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


def _err():
    return lib().orc_last_error().decode()


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _state(U, n):
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.shape != (n, 6):
        raise ValueError(f"expected state of shape ({n}, 6), got {U.shape}")
    return U


class Mesh:
    """Balanced octree mesh built by the oracle (Sec. 4)."""

    def __init__(self, trees=(1, 1, 1), level_min=0, level_max=0, phi0=None, band=0.9,
                 leaves=None):
        L = lib()
        T = (C.c_int32 * 3)(*trees)
        self._cb = None
        if phi0 is not None:
            def cb(xyz, n, out, user, _f=phi0):
                pts = np.ctypeslib.as_array(xyz, shape=(n, 3))
                res = np.ctypeslib.as_array(out, shape=(n,))
                res[:] = _f(pts)
            self._cb = PHI0_FN(cb)
        else:
            self._cb = PHI0_FN()
        lv = None
        nl = 0
        if leaves is not None:
            leaves = np.ascontiguousarray(leaves, dtype=np.int32).reshape(-1, 4)
            lv = leaves.ctypes.data_as(C.POINTER(C.c_int32))
            nl = leaves.shape[0]
        h = C.c_void_p()
        rc = L.orc_mesh_build(T, level_min, level_max, self._cb, None, band, lv, nl, C.byref(h))
        if rc != 0:
            raise ValueError("oracle mesh build failed: " + _err())
        self._h = h
        s = (C.c_int64 * 5)()
        L.orc_mesh_sizes(h, s)
        E, n, nh, nc, D = (int(v) for v in s)
        self.trees = tuple(trees)
        self.level_max = D
        self.leaves = np.zeros((E, 4), np.int32)
        self.elem = np.zeros((E, 8), np.int32)
        self.nodes = np.zeros((n, 3), np.int32)
        self.bflags = np.zeros(n, np.uint8)
        self.hang_xyz = np.zeros((nh, 3), np.int32)
        self.hang_off = np.zeros(nh + 1, np.int64)
        self.hang_ids = np.zeros(nc, np.int32)
        self.hang_w = np.zeros(nc, np.float64)
        L.orc_mesh_arrays(h, self.leaves.ctypes.data, self.elem.ctypes.data,
                          self.nodes.ctypes.data, self.bflags.ctypes.data,
                          self.hang_xyz.ctypes.data, self.hang_off.ctypes.data,
                          self.hang_ids.ctypes.data, self.hang_w.ctypes.data)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_mesh_free(h)
            self._h = None

    @property
    def n_nodes(self):
        return self.nodes.shape[0]

    @property
    def n_leaves(self):
        return self.leaves.shape[0]

    def node_xyz(self):
        """Physical coordinates of the independent nodes."""
        return self.nodes.astype(np.float64) * 2.0 ** (-self.level_max)

    def residual(self, p, block, Unew, Uold, forcing=None, bc=None):
        """Block residual; forcing (E, 8, 6) at the Gauss points, bc (n, 6)
        whose boundary velocities are the wall data at t^{k+1}."""
        n = self.n_nodes
        Unew, Uold = _state(Unew, n), _state(Uold, n)
        R = np.zeros((n, 6))
        if forcing is not None:
            forcing = np.ascontiguousarray(forcing, dtype=np.float64)
            assert forcing.shape == (self.n_leaves, 8, 6)
        if bc is not None:
            bc = _state(bc, n)
        rc = lib().orc_residual(self._h, C.byref(p), block, _dp(Unew), _dp(Uold), _dp(forcing),
                                _dp(bc), _dp(R))
        if rc != 0:
            raise RuntimeError(_err())
        return R

    def jvp(self, p, block, Unew, Uold, dU):
        n = self.n_nodes
        Unew, Uold, dU = _state(Unew, n), _state(Uold, n), _state(dU, n)
        out = np.zeros((n, 6))
        rc = lib().orc_jvp(self._h, C.byref(p), block, _dp(Unew), _dp(Uold), _dp(dU), _dp(out))
        if rc != 0:
            raise RuntimeError(_err())
        return out

    def jvp_full(self, p, block, Unew, Uold, dU):
        """The block's rows of the coupled Jacobian applied to dU (all six fields)."""
        n = self.n_nodes
        Unew, Uold, dU = _state(Unew, n), _state(Uold, n), _state(dU, n)
        out = np.zeros((n, 6))
        rc = lib().orc_jvp_full(self._h, C.byref(p), block, _dp(Unew), _dp(Uold), _dp(dU), _dp(out))
        if rc != 0:
            raise RuntimeError(_err())
        return out

    def residual_rows(self, p, block, Unew, Uold, rows, dU=None):
        """Residual (dU None) or JVP rows of the listed nodes only."""
        n = self.n_nodes
        Unew, Uold = _state(Unew, n), _state(Uold, n)
        if dU is not None:
            dU = _state(dU, n)
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.zeros((rows.shape[0], 6))
        rc = lib().orc_residual_rows(self._h, C.byref(p), block, _dp(Unew), _dp(Uold),
                                     rows.ctypes.data_as(C.POINTER(C.c_int32)), rows.shape[0],
                                     _dp(dU), _dp(out))
        if rc != 0:
            raise RuntimeError(_err())
        return out

    def diag_blocks(self, p, block, Unew, Uold):
        n = self.n_nodes
        nf = 2 if block == BLOCK_CH else 4
        Unew, Uold = _state(Unew, n), _state(Uold, n)
        out = np.zeros((n, nf, nf))
        rc = lib().orc_diag_blocks(self._h, C.byref(p), block, _dp(Unew), _dp(Uold), _dp(out))
        if rc != 0:
            raise RuntimeError(_err())
        return out

    def diagnostics(self, p, U):
        U = _state(U, self.n_nodes)
        m, e = C.c_double(), C.c_double()
        lib().orc_diagnostics(self._h, C.byref(p), _dp(U), C.byref(m), C.byref(e))
        return m.value, e.value

    def step(self, p, opts, U, forcing=None, bc=None):
        """One CN step from U; forcing (E, 8, 6) at the Gauss points at
        t^{k+1/2}, bc (n, 6) with the wall velocities at t^{k+1}."""
        U = _state(U, self.n_nodes).copy()
        st = StepStats()
        if forcing is not None:
            forcing = np.ascontiguousarray(forcing, dtype=np.float64)
            assert forcing.shape == (self.n_leaves, 8, 6)
        if bc is not None:
            bc = _state(bc, self.n_nodes)
        rc = lib().orc_step(self._h, C.byref(p), C.byref(opts), _dp(U), _dp(forcing), _dp(bc),
                            C.byref(st))
        if rc != 0:
            raise RuntimeError(_err())
        return U, st

    def qp_coords(self):
        """Physical coordinates of the 2x2x2 Gauss points, shape (E, 8, 3), in
        the oracle's point order q = i + 2j + 4k."""
        g = 1.0 / np.sqrt(3.0)
        s = np.array([[-1 if not (q >> d) & 1 else 1 for d in range(3)] for q in range(8)], float)
        unit = 2.0 ** (-self.level_max)
        x0 = self.leaves[:, :3].astype(np.float64) * unit
        h = 2.0 ** (-self.leaves[:, 3].astype(np.float64))
        return x0[:, None, :] + 0.5 * h[:, None, None] * (1.0 + s[None, :, :] * g)

    def q2(self):
        """The cG(2) numbering of this mesh (27-node leaves)."""
        return MeshQ2(self)


class MeshQ2:
    """Triquadratic numbering on the leaves of an oracle Mesh: node a = i +
    3j + 9k of a leaf at its anchor plus (i, j, k) half sides; coordinates in
    doubled units 2^-(level_max+1).  Hanging lattice points take the
    coarsest neighbouring leaf's triquadratic interpolant (Sec. 4, carried
    over to cG(2)).  Both blocks' rows (CH and VMS NS) on this space."""

    def __init__(self, mesh):
        L = lib()
        self.mesh = mesh
        h = C.c_void_p()
        if L.orc_q2_build(mesh._h, C.byref(h)) != 0:
            raise ValueError("oracle Q2 numbering failed: " + _err())
        self._h = h
        s = (C.c_int64 * 3)()
        L.orc_q2_sizes(h, s)
        n, nh, nc = (int(v) for v in s)
        E = mesh.n_leaves
        self.elem = np.zeros((E, 27), np.int32)
        self.nodes = np.zeros((n, 3), np.int32)
        self.hang_xyz = np.zeros((nh, 3), np.int32)
        self.hang_off = np.zeros(nh + 1, np.int64)
        self.hang_ids = np.zeros(nc, np.int32)
        self.hang_w = np.zeros(nc, np.float64)
        self.bflags = np.zeros(n, np.uint8)
        L.orc_q2_arrays(h, self.elem.ctypes.data, self.nodes.ctypes.data, self.hang_xyz.ctypes.data,
                        self.hang_off.ctypes.data, self.hang_ids.ctypes.data, self.hang_w.ctypes.data,
                        self.bflags.ctypes.data)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_q2_free(h)
            self._h = None

    @property
    def n_nodes(self):
        return self.nodes.shape[0]

    def node_xyz(self):
        """Physical coordinates of the independent nodes."""
        return self.nodes.astype(np.float64) * 2.0 ** (-(self.mesh.level_max + 1))

    def hang_coords(self):
        return self.hang_xyz.astype(np.float64) * 2.0 ** (-(self.mesh.level_max + 1))

    def residual(self, p, Unew, Uold, block=BLOCK_CH):
        """Block rows over the Q2 nodes: CH fields 0, 1 or NS fields 2..5."""
        n = self.n_nodes
        Unew, Uold = _state(Unew, n), _state(Uold, n)
        R = np.zeros((n, 6))
        if lib().orc_q2_residual(self.mesh._h, self._h, C.byref(p), block, _dp(Unew), _dp(Uold),
                                 _dp(R)) != 0:
            raise RuntimeError(_err())
        return R

    def jvp(self, p, Unew, Uold, dU, block=BLOCK_CH):
        """The block's Jacobian (derivative in its own unknowns) applied to dU."""
        n = self.n_nodes
        Unew, Uold, dU = _state(Unew, n), _state(Uold, n), _state(dU, n)
        out = np.zeros((n, 6))
        if lib().orc_q2_jvp(self.mesh._h, self._h, C.byref(p), block, _dp(Unew), _dp(Uold), _dp(dU),
                            _dp(out)) != 0:
            raise RuntimeError(_err())
        return out
