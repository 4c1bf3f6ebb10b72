"""ctypes wrapper of the FP64 reference library (oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The HIP product path never does.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_D2Q9 = os.path.join(HERE, "liboracle_d2q9.so")  # the same source built for the paper's D2Q9

UNIFORM, WEIGHTED, BOUNCEBACK, STOCHASTIC = 0, 1, 2, 3
PASSIVE, BARYCENTRIC = 0, 1
XPERIODIC, XRESERVOIR, XINFLOW = 0, 1, 2


def build(force=True):
    """Compile oracle.c with gcc (plain C, OpenMP, no FMA contraction), once
    for D3Q19 and once for D2Q9."""
    for path, extra in ((LIB, []), (LIB_D2Q9, ["-DORC_D2Q9"])):
        if not force and os.path.exists(path):
            continue
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", *extra, "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [("tau_gas", ctypes.c_double), ("tau_species", ctypes.c_double),
                ("p", ctypes.c_double), ("p_stick", ctypes.c_double),
                ("c_inlet", ctypes.c_double), ("rho0", ctypes.c_double), ("c0", ctypes.c_double),
                ("force", ctypes.c_double * 3),
                ("sputter", ctypes.c_int32), ("coupling", ctypes.c_int32),
                ("species_x", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("p_stick_product", ctypes.c_double),
                ("product", ctypes.c_int32), ("pad2", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("wall_diffuse", ctypes.c_double)]


_libs = {}
LATTICES = {"D3Q19": LIB, "D2Q9": LIB_D2Q9}


def lib(lattice="D3Q19"):
    """The oracle library of one velocity set (D3Q19 default, or D2Q9)."""
    if lattice not in _libs:
        path = LATTICES[lattice]
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.POINTER(Params)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        for name in ("orc_fields",):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]
        L.orc_conversion_map.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_totals.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_step_count.argtypes = [ctypes.c_void_p]
        L.orc_step_count.restype = ctypes.c_long
        L.orc_get_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_set_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_get_state_product.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_set_state_product.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_product.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_product_flux.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_link_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_d3q19.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_d3q19.restype = ctypes.c_int
        L.orc_wall_sigma_from_kn.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_int)]
        L.orc_wall_sigma_from_kn.restype = ctypes.c_double
        for name in ("orc_kn_from_tau", "orc_tau_from_kn", "orc_da_from_p"):
            getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_double]
            getattr(L, name).restype = ctypes.c_double
        L.orc_p_from_da.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.orc_p_from_da.restype = ctypes.c_double
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_guo_source.argtypes = [ctypes.c_double, dp, dp, dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _libs[lattice] = L
    return _libs[lattice]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def d3q19(lattice="D3Q19"):
    """(c, w, opp) of the oracle's velocity set (D3Q19, or D2Q9 with lattice="D2Q9")."""
    q = 19 if lattice == "D3Q19" else 9
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, dtype=np.int32)
    assert lib(lattice).orc_d3q19(c.ctypes.data, w.ctypes.data, opp.ctypes.data) == q
    return c, w, opp


def kn_from_tau(tau, delta):
    return lib().orc_kn_from_tau(tau, delta)


def tau_from_kn(kn, delta):
    return lib().orc_tau_from_kn(kn, delta)


def wall_sigma_from_kn(kn, delta, accommodation=1.0):
    """(sigma, clamped): diffuse fraction of the gas wall that gives Maxwell's
    first-order slip at kn (orc_wall_sigma_from_kn)."""
    cl = ctypes.c_int(0)
    s = lib().orc_wall_sigma_from_kn(kn, delta, accommodation, ctypes.byref(cl))
    return s, bool(cl.value)


def p_from_da(da, delta):
    cl = ctypes.c_int(0)
    p = lib().orc_p_from_da(da, delta, ctypes.byref(cl))
    return p, bool(cl.value)


def da_from_p(p, delta):
    return lib().orc_da_from_p(p, delta)


def equilibrium(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib().orc_equilibrium(rho, _dp(u), _dp(out))
    return out


def guo_source(tau, u, F):
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().orc_guo_source(tau, _dp(u), _dp(F), _dp(out))
    return out


def philox4x32_10(ctr, key):
    """The oracle's Philox4x32-10 on one counter (4 words) and key (2 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def threads():
    return lib().orc_threads()


def set_threads(n):
    """Threads of the oracle's parallel loops from now on (results are the
    same for any count)."""
    lib().orc_set_threads(int(n))


class Oracle:
    """One FP64 reference simulation of the gas + reactant lattices, plus the
    product lattice when `product` is set (p_stick_product = p_S^P)."""

    def __init__(self, vox, tau=(0.8, 0.7), p=0.1, p_stick=0.95, c_inlet=1.0, rho0=1.0, c0=0.0,
                 force=(0.0, 0.0, 0.0), sputter=UNIFORM, coupling=PASSIVE, species_x=XRESERVOIR,
                 product=False, p_stick_product=0.0, seed=0, wall_diffuse=0.0, lattice="D3Q19"):
        vox = np.ascontiguousarray(vox, dtype=np.uint8)
        assert vox.ndim == 3
        self.nz, self.ny, self.nx = vox.shape
        if lattice == "D2Q9" and self.nz != 1:
            raise ValueError("D2Q9 runs on one z-plane (nz = 1)")
        self.lattice = lattice
        self.q = 19 if lattice == "D3Q19" else 9
        self._L = lib(lattice)
        self.n = vox.size
        self.vox = vox
        prm = Params()
        prm.tau_gas, prm.tau_species = float(tau[0]), float(tau[1])
        prm.p, prm.p_stick, prm.c_inlet = float(p), float(p_stick), float(c_inlet)
        prm.rho0, prm.c0 = float(rho0), float(c0)
        for a in range(3):
            prm.force[a] = float(force[a])
        prm.sputter, prm.coupling, prm.species_x = int(sputter), int(coupling), int(species_x)
        prm.product, prm.p_stick_product = int(bool(product)), float(p_stick_product)
        prm.seed = int(seed)
        prm.wall_diffuse = float(wall_diffuse)
        self.params = prm
        h = self._L.orc_create(self.nx, self.ny, self.nz, vox.ctypes.data, ctypes.byref(prm))
        if not h:
            raise MemoryError("orc_create failed")
        self._h = h

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._L.orc_step(self._h, int(n))

    @property
    def step_count(self):
        return self._L.orc_step_count(self._h)

    def fields(self):
        shape = (self.nz, self.ny, self.nx)
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        c = np.zeros(self.n)
        self._L.orc_fields(self._h, rho.ctypes.data, u.ctypes.data, c.ctypes.data)
        return rho.reshape(shape), u.reshape((3,) + shape), c.reshape(shape)

    def conversion_map(self):
        out = np.zeros(self.n)
        self._L.orc_conversion_map(self._h, out.ctypes.data)
        return out.reshape((self.nz, self.ny, self.nx))

    def totals(self):
        t = np.zeros(6)
        self._L.orc_totals(self._h, t.ctypes.data)
        keys = ("mass_gas", "mass_species", "converted", "lost", "influx", "outflux")
        return dict(zip(keys, t.tolist()))

    def product(self):
        """(rho_P field, totals dict, stuck map p_S^P sum_t In_P(k, t))."""
        shape = (self.nz, self.ny, self.nx)
        c = np.zeros(self.n)
        t = np.zeros(4)
        st = np.zeros(self.n)
        self._L.orc_product(self._h, c.ctypes.data, t.ctypes.data, st.ctypes.data)
        keys = ("mass_product", "lost_product", "product_out_inlet", "product_out_outlet")
        return c.reshape(shape), dict(zip(keys, t.tolist())), st.reshape(shape)

    def product_flux(self):
        """Phi_P(x): sum over each cross-section of rho_P u_x."""
        phi = np.zeros(self.nx)
        self._L.orc_product_flux(self._h, phi.ctypes.data)
        return phi

    def get_state_product(self):
        fP = np.zeros((self.n, self.q))
        self._L.orc_get_state_product(self._h, fP.ctypes.data)
        return fP

    def set_state_product(self, fP):
        a = np.ascontiguousarray(fP, dtype=np.float64)
        self._L.orc_set_state_product(self._h, a.ctypes.data)

    def link_counts(self):
        b = np.zeros(self.n, dtype=np.uint8)
        self._L.orc_link_counts(self._h, b.ctypes.data)
        return b.reshape((self.nz, self.ny, self.nx))

    def get_state(self):
        fC = np.zeros((self.n, self.q))
        fR = np.zeros((self.n, self.q))
        self._L.orc_get_state(self._h, fC.ctypes.data, fR.ctypes.data)
        return fC, fR

    def set_state(self, fC=None, fR=None):
        a = None if fC is None else np.ascontiguousarray(fC, dtype=np.float64)
        b = None if fR is None else np.ascontiguousarray(fR, dtype=np.float64)
        self._L.orc_set_state(self._h, None if a is None else a.ctypes.data,
                            None if b is None else b.ctypes.data)
