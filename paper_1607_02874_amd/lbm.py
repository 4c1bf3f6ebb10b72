"""Thin ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP library liblbm.so; this module only
converts Python/numpy/torch arguments to the C structs and pointers.  There is
no fallback: if the library is missing or cannot load, importing the binding
raises.  PyTorch, when present, provides device memory (its caching allocator
through the lbm_device hooks) and the stream work is queued on.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_ENONFINITE, LBM_EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "LBM_OK", 1: "LBM_EINVAL", 2: "LBM_ENOMEM", 3: "LBM_EDEVICE", 4: "LBM_ESTATE",
                5: "LBM_ENONFINITE", 6: "LBM_EUNSUPPORTED"}
FLUID, INERT, CATALYTIC = 0, 1, 2
SPUTTER_UNIFORM, SPUTTER_WEIGHTED, SPUTTER_BOUNCEBACK, SPUTTER_STOCHASTIC = 0, 1, 2, 3
COUPLE_PASSIVE, COUPLE_BARYCENTRIC = 0, 1
XBC_PERIODIC, XBC_RESERVOIR, XBC_INFLOW = 0, 1, 2
STORE_F32, STORE_F16, STORE_BF16, STORE_F64 = 0, 1, 2, 3
ROUND_NEAREST, ROUND_STOCHASTIC = 0, 1
LATTICE_D3Q19, LATTICE_D2Q9 = 0, 1
TUNE_YTILE, TUNE_SWEEP, TUNE_EMISSION = 0, 1, 2
STORAGE_BYTES = {STORE_F32: 4, STORE_F16: 2, STORE_BF16: 2, STORE_F64: 8}
STORAGE_NAMES = {STORE_F32: "f32", STORE_F16: "f16", STORE_BF16: "bf16", STORE_F64: "f64"}
# Direction numbering of lbm_populations (as documented in include/lbm.h).
D3Q19 = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1),
                  (0, 1, 1), (0, 1, -1)] + [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (-1, -1, 0), (-1, 1, 0),
                                            (-1, 0, -1), (-1, 0, 1), (0, -1, -1), (0, -1, 1)], dtype=np.int64)


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lbm_geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("voxels", ctypes.c_void_p), ("pore_size", ctypes.c_double)]


class lbm_bc(ctypes.Structure):
    _fields_ = [("sputter", ctypes.c_int32), ("coupling", ctypes.c_int32), ("species_x", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("p_stick", ctypes.c_double), ("c_inlet", ctypes.c_double),
                ("rho0", ctypes.c_double), ("c0", ctypes.c_double), ("c_ref", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("product", ctypes.c_int32), ("rounding", ctypes.c_int32),
                ("p_stick_product", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("wall_diffuse", ctypes.c_double), ("wall_accommodation", ctypes.c_double),
                ("lattice", ctypes.c_int32), ("reserved_bc", ctypes.c_int32), ("store_ux", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class lbm_device(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class lbm_totals_t(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass_gas", ctypes.c_double), ("mass_species", ctypes.c_double),
                ("converted", ctypes.c_double), ("lost", ctypes.c_double), ("influx", ctypes.c_double),
                ("outflux", ctypes.c_double), ("nonfinite", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mass_product", ctypes.c_double), ("lost_product", ctypes.c_double),
                ("product_out_inlet", ctypes.c_double), ("product_out_outlet", ctypes.c_double)]


class lbm_info(ctypes.Structure):
    _fields_ = [("tau_gas", ctypes.c_double), ("tau_species", ctypes.c_double), ("kn", ctypes.c_double),
                ("p", ctypes.c_double), ("da", ctypes.c_double), ("pore_size", ctypes.c_double),
                ("p_clamped", ctypes.c_int32), ("storage", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("n_fluid", ctypes.c_int64), ("n_interface", ctypes.c_int64),
                ("n_catalytic_links", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("wall_sigma", ctypes.c_double), ("wall_clamped", ctypes.c_int32), ("reserved_info", ctypes.c_int32)]


class lbm_kernel_times_t(ctypes.Structure):
    _fields_ = [("ms_sweep", ctypes.c_double), ("ms_interface", ctypes.c_double), ("ms_xflux", ctypes.c_double),
                ("ms_reduce", ctypes.c_double), ("n_sweep", ctypes.c_int64), ("n_interface", ctypes.c_int64),
                ("n_xflux", ctypes.c_int64), ("n_reduce", ctypes.c_int64)]


def _load():
    # One HIP runtime per process: PyTorch bundles its own libamdhip64 with the
    # same soname as the system one.  Loading torch first makes liblbm.so bind
    # to the runtime torch already holds, so the library can share torch's
    # device memory and streams; without torch the system runtime is used.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run "
                          "`python -m paper_1607_02874_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    ctx = ctypes.c_void_p
    st = ctypes.c_int
    sig = {
        "lbm_create": (st, [P(lbm_geometry), ctypes.c_double, ctypes.c_double, P(ctypes.c_double), P(lbm_bc),
                            P(ctx)]),
        "lbm_create_on": (st, [P(lbm_geometry), ctypes.c_double, ctypes.c_double, P(ctypes.c_double), P(lbm_bc),
                               P(lbm_device), P(ctx)]),
        "lbm_step": (st, [ctx, ctypes.c_int64]),
        "lbm_inspect": (st, [P(lbm_geometry), ctypes.c_double, ctypes.c_double, P(ctypes.c_double), P(lbm_bc),
                             P(lbm_info)]),
        "lbm_fields": (st, [ctx, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_fields_device": (st, [ctx, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_fields_noalloc": (st, [ctx, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_stream_copy": (st, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
        "lbm_stream_pull": (st, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_void_p]),
        "lbm_conversion_map": (st, [ctx, ctypes.c_void_p]),
        "lbm_product_fields": (st, [ctx, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_populations": (st, [ctx, P(ctypes.c_int32), P(ctypes.c_int32), ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_totals": (st, [ctx, P(lbm_totals_t)]),
        "lbm_query": (st, [ctx, P(lbm_info)]),
        "lbm_active_links": (st, [ctx, ctypes.c_void_p]),
        "lbm_synchronize": (st, [ctx]),
        "lbm_set_timing": (st, [ctx, ctypes.c_int32]),
        "lbm_set_tunable": (st, [ctx, ctypes.c_int32, ctypes.c_int64]),
        "lbm_get_tunable": (st, [ctx, ctypes.c_int32, P(ctypes.c_int64)]),
        "lbm_kernel_times": (st, [ctx, P(lbm_kernel_times_t)]),
        "lbm_autotune": (st, [ctx, ctypes.c_int32, P(ctypes.c_double)]),
        "lbm_batch_autotune": (st, [ctx, ctypes.c_int32, P(ctypes.c_double)]),
        "lbm_save": (st, [ctx, ctypes.c_char_p]),
        "lbm_load": (st, [ctx, ctypes.c_char_p]),
        "lbm_last_error": (ctypes.c_char_p, [ctx]),
        "lbm_destroy": (None, [ctx]),
        "lbm_batch_create": (st, [ctypes.c_int32, P(lbm_geometry), P(ctypes.c_double), P(ctypes.c_double),
                                  P(ctypes.c_double), P(lbm_bc), P(lbm_device), P(ctx)]),
        "lbm_batch_step": (st, [ctx, ctypes.c_int64]),
        "lbm_batch_fields": (st, [ctx, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_batch_conversion_map": (st, [ctx, ctypes.c_int32, ctypes.c_void_p]),
        "lbm_batch_totals": (st, [ctx, ctypes.c_int32, P(lbm_totals_t)]),
        "lbm_batch_query": (st, [ctx, ctypes.c_int32, P(lbm_info)]),
        "lbm_batch_synchronize": (st, [ctx]),
        "lbm_batch_set_graph": (st, [ctx, ctypes.c_int32]),
        "lbm_batch_set_timing": (st, [ctx, ctypes.c_int32]),
        "lbm_batch_kernel_times": (st, [ctx, P(lbm_kernel_times_t)]),
        "lbm_batch_set_tunable": (st, [ctx, ctypes.c_int32, ctypes.c_int64]),
        "lbm_batch_get_tunable": (st, [ctx, ctypes.c_int32, P(ctypes.c_int64)]),
        "lbm_batch_last_error": (ctypes.c_char_p, [ctx]),
        "lbm_batch_destroy": (None, [ctx]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_LIB = _load()


def library():
    return _LIB


def header_functions(path=HEADER):
    """Names of the functions include/lbm.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(lbm_[a-z_]+)\s*\(", text, flags=re.M)))


def _check(status, ctx=None):
    if status != LBM_OK:
        msg = _LIB.lbm_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")


def _bcheck(status, batch=None):
    if status != LBM_OK:
        msg = _LIB.lbm_batch_last_error(batch)
        raise LbmError(status, msg.decode() if msg else "")


def _ptr(a):
    """Data pointer of a numpy array or torch tensor (None passes NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


class _TorchDevice:
    """lbm_device hooks backed by the PyTorch caching allocator and stream."""

    def __init__(self, stream=None):
        import torch

        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = lbm_device(ctypes.c_void_p(self.stream.cuda_stream), self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:
            return None

    def _do_free(self, ptr, user):
        self.torch.cuda.caching_allocator_delete(ptr)


def _geometry(vox, pore_size):
    vox = np.ascontiguousarray(vox, dtype=np.uint8)
    if vox.ndim != 3:
        raise ValueError("vox must be (nz, ny, nx)")
    nz, ny, nx = vox.shape
    return vox, lbm_geometry(nx, ny, nz, 0, vox.ctypes.data, float(pore_size))


def _bc(sputter=SPUTTER_UNIFORM, coupling=COUPLE_PASSIVE, species_x=XBC_RESERVOIR, storage=STORE_F32,
        p_stick=0.95, c_inlet=1.0, rho0=1.0, c0=0.0, c_ref=-1.0, force=(0.0, 0.0, 0.0), product=False,
        p_stick_product=0.0, seed=0, wall_diffuse=0.0, rounding=ROUND_NEAREST, wall_accommodation=0.0,
        lattice=LATTICE_D3Q19, store_ux=0.0):
    return lbm_bc(int(sputter), int(coupling), int(species_x), int(storage), float(p_stick), float(c_inlet),
                  float(rho0), float(c0), float(c_ref), (ctypes.c_double * 3)(*[float(f) for f in force]),
                  int(bool(product)), int(rounding), float(p_stick_product), int(seed), float(wall_diffuse),
                  float(wall_accommodation), int(lattice), 0, float(store_ux))


def lbm_create(vox, da, tau=(0.0, 0.0), kn=0.0, pore_size=1.0, device=None, **bc_kw):
    """Call lbm_create_on.  vox is a (nz, ny, nx) uint8 array; device is an
    lbm_device struct holder (see use_torch) or None for hipMalloc and the
    null stream; bc_kw are the lbm_bc fields (sputter, coupling, species_x,
    storage, p_stick, c_inlet, rho0, c0, c_ref, force, product,
    p_stick_product, seed, wall_diffuse, rounding, wall_accommodation, lattice, store_ux).  Returns the raw
    context handle."""
    vox, g = _geometry(vox, pore_size)
    bc = _bc(**bc_kw)
    t = (ctypes.c_double * 2)(float(tau[0]), float(tau[1]))
    out = ctypes.c_void_p()
    dev = ctypes.byref(device.struct) if device is not None else None
    _check(_LIB.lbm_create_on(ctypes.byref(g), float(kn), float(da), t, ctypes.byref(bc), dev,
                              ctypes.byref(out)))
    return out


def inspect(vox, da, tau=(0.0, 0.0), kn=0.0, pore_size=1.0, **bc_kw):
    """lbm_inspect: parameter maps, node/interface/link counts and planned
    device bytes of a context, computed on the host (no GPU needed)."""
    vox, g = _geometry(vox, pore_size)
    bc = _bc(**bc_kw)
    t = (ctypes.c_double * 2)(float(tau[0]), float(tau[1]))
    info = lbm_info()
    _check(_LIB.lbm_inspect(ctypes.byref(g), float(kn), float(da), t, ctypes.byref(bc), ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in lbm_info._fields_}


class Sim:
    """One context: the carrier and reactant lattices over a voxel map.

    Keyword arguments are the lbm_bc fields (see _bc).  Options beyond the
    default method: product=True with p_stick_product (the product lattice;
    product_fields() and the product totals), sputter=SPUTTER_STOCHASTIC with
    seed (random sputtering matrix), wall_diffuse=sigma (diffuse carrier
    wall) or wall_accommodation=sigma_v (the diffuse fraction derived from Kn
    for Maxwell's slip; info()["wall_sigma"] reports it),
    rounding=ROUND_STOCHASTIC (stochastic rounding of 16-bit stores),
    store_ux=U (a reference flow: the carrier is stored and relaxed as its
    deviation less the part linear in the x-velocity U),
    lattice=LATTICE_D2Q9 (the paper's D2Q9 on one plane, FP64; see lbm.h)."""

    def __init__(self, vox, da, tau=(0.0, 0.0), kn=0.0, pore_size=1.0, use_torch=True, stream=None, **kw):
        self._h = None
        self._device = None
        if use_torch:
            import torch

            if torch.cuda.is_available():
                self._device = _TorchDevice(stream)
        self.shape = tuple(np.shape(vox))
        self.n = int(np.prod(self.shape))
        self._h = lbm_create(vox, da, tau=tau, kn=kn, pore_size=pore_size, device=self._device, **kw)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _LIB.lbm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n=1):
        _check(_LIB.lbm_step(self._h, int(n)), self._h)

    def synchronize(self):
        _check(_LIB.lbm_synchronize(self._h), self._h)

    def fields(self):
        """(rho, u, conc) as float64 numpy arrays, u of shape (3, nz, ny, nx)."""
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        c = np.zeros(self.n)
        _check(_LIB.lbm_fields(self._h, rho.ctypes.data, u.ctypes.data, c.ctypes.data), self._h)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape), c.reshape(self.shape)

    def fields_noalloc(self):
        """fields() through lbm_fields_noalloc (no device allocation)."""
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        c = np.zeros(self.n)
        _check(_LIB.lbm_fields_noalloc(self._h, rho.ctypes.data, u.ctypes.data, c.ctypes.data), self._h)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape), c.reshape(self.shape)

    def fields_device(self, rho=None, u=None, conc=None):
        """Write float32 fields into device tensors (any may be None)."""
        _check(_LIB.lbm_fields_device(self._h, _ptr(rho), _ptr(u), _ptr(conc)), self._h)

    def populations(self, origin=(0, 0, 0), extent=None):
        """Pre-collision populations (fC, fR) of the box origin (x, y, z) and
        extent (wx, wy, wz), each float64 of shape (19, wz, wy, wx) in the
        library's direction numbering (D3Q19 below)."""
        nz, ny, nx = self.shape
        if extent is None:
            extent = (nx - origin[0], ny - origin[1], nz - origin[2])
        o = (ctypes.c_int32 * 3)(*[int(v) for v in origin])
        e = (ctypes.c_int32 * 3)(*[int(v) for v in extent])
        shape = (19, int(extent[2]), int(extent[1]), int(extent[0]))
        fC = np.zeros(shape)
        fR = np.zeros(shape)
        _check(_LIB.lbm_populations(self._h, o, e, fC.ctypes.data, fR.ctypes.data), self._h)
        return fC, fR

    def conversion_map(self):
        out = np.zeros(self.n)
        _check(_LIB.lbm_conversion_map(self._h, out.ctypes.data), self._h)
        return out.reshape(self.shape)

    def product_fields(self):
        """lbm_product_fields: (rho_P field, stuck-product map, Phi_P(x))."""
        conc = np.zeros(self.n)
        stuck = np.zeros(self.n)
        phi = np.zeros(self.shape[2])
        _check(_LIB.lbm_product_fields(self._h, conc.ctypes.data, stuck.ctypes.data, phi.ctypes.data), self._h)
        return conc.reshape(self.shape), stuck.reshape(self.shape), phi

    def totals(self):
        t = lbm_totals_t()
        _check(_LIB.lbm_totals(self._h, ctypes.byref(t)), self._h)
        return {k: getattr(t, k) for k, _ in lbm_totals_t._fields_ if k != "reserved"}

    def info(self):
        i = lbm_info()
        _check(_LIB.lbm_query(self._h, ctypes.byref(i)), self._h)
        return {k: getattr(i, k) for k, _ in lbm_info._fields_}

    def active_links(self):
        b = np.zeros(self.n, dtype=np.uint8)
        _check(_LIB.lbm_active_links(self._h, b.ctypes.data), self._h)
        return b.reshape(self.shape)

    def set_tunable(self, which, value):
        _check(_LIB.lbm_set_tunable(self._h, int(which), int(value)), self._h)

    def get_tunable(self, which):
        v = ctypes.c_int64()
        _check(_LIB.lbm_get_tunable(self._h, int(which), ctypes.byref(v)), self._h)
        return v.value

    def set_timing(self, on=True):
        """True or 1: time every launch; 2: the sweep only; False or 0: off."""
        level = 1 if on is True else (0 if on is False else int(on))
        _check(_LIB.lbm_set_timing(self._h, level), self._h)

    def autotune(self, reps=5):
        """Time the sweep for every launch-shape candidate and keep the
        fastest (state unchanged).  Returns the winner's mean sweep time (ms)."""
        ms = ctypes.c_double()
        _check(_LIB.lbm_autotune(self._h, int(reps), ctypes.byref(ms)), self._h)
        return ms.value

    def kernel_times(self):
        t = lbm_kernel_times_t()
        _check(_LIB.lbm_kernel_times(self._h, ctypes.byref(t)), self._h)
        return {k: getattr(t, k) for k, _ in lbm_kernel_times_t._fields_}

    def save(self, path):
        _check(_LIB.lbm_save(self._h, str(path).encode()), self._h)

    def load(self, path):
        _check(_LIB.lbm_load(self._h, str(path).encode()), self._h)


class Batch:
    """Many independent samples advanced together (lbm_batch_*).  samples is
    a list of dicts with the arguments of Sim: vox, da, and optionally tau,
    kn, pore_size and the lbm_bc fields; storage, sputter, coupling and
    species_x must be the same in all."""

    def __init__(self, samples, use_torch=True, stream=None, graph=False):
        self._h = None
        self._device = None
        if use_torch:
            import torch

            if torch.cuda.is_available():
                self._device = _TorchDevice(stream)
        n = len(samples)
        self.shapes = []
        keep = []
        geoms = (lbm_geometry * n)()
        bcs = (lbm_bc * n)()
        kn = (ctypes.c_double * n)()
        da = (ctypes.c_double * n)()
        tau = (ctypes.c_double * (2 * n))()
        for i, smp in enumerate(samples):
            smp = dict(smp)
            vox, g = _geometry(smp.pop("vox"), smp.pop("pore_size", 1.0))
            keep.append(vox)
            self.shapes.append(vox.shape)
            geoms[i] = g
            da[i] = float(smp.pop("da"))
            kn[i] = float(smp.pop("kn", 0.0))
            t = smp.pop("tau", (0.0, 0.0))
            tau[2 * i], tau[2 * i + 1] = float(t[0]), float(t[1])
            bcs[i] = _bc(**smp)
        out = ctypes.c_void_p()
        dev = ctypes.byref(self._device.struct) if self._device is not None else None
        _bcheck(_LIB.lbm_batch_create(n, geoms, kn, da, tau, bcs, dev, ctypes.byref(out)))
        self._h = out
        self.n = n
        if graph:
            self.set_graph(True)

    def close(self):
        if self._h is not None and self._h.value:
            _LIB.lbm_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n=1):
        _bcheck(_LIB.lbm_batch_step(self._h, int(n)), self._h)

    def synchronize(self):
        _bcheck(_LIB.lbm_batch_synchronize(self._h), self._h)

    def set_graph(self, on=True):
        _bcheck(_LIB.lbm_batch_set_graph(self._h, 1 if on else 0), self._h)

    def set_tunable(self, which, value):
        _bcheck(_LIB.lbm_batch_set_tunable(self._h, int(which), int(value)), self._h)

    def set_timing(self, on=True):
        """Events around every batched sweep (steps then run without graphs)."""
        _bcheck(_LIB.lbm_batch_set_timing(self._h, 2 if on else 0), self._h)

    def kernel_times(self):
        t = lbm_kernel_times_t()
        _bcheck(_LIB.lbm_batch_kernel_times(self._h, ctypes.byref(t)), self._h)
        return {"ms_sweep": t.ms_sweep, "n_sweep": t.n_sweep}

    def autotune(self, reps=5):
        ms = ctypes.c_double()
        _bcheck(_LIB.lbm_batch_autotune(self._h, int(reps), ctypes.byref(ms)), self._h)
        return ms.value

    def get_tunable(self, which):
        v = ctypes.c_int64()
        _bcheck(_LIB.lbm_batch_get_tunable(self._h, int(which), ctypes.byref(v)), self._h)
        return v.value

    def fields(self, i):
        shape = self.shapes[i]
        nn = int(np.prod(shape))
        rho, u, c = np.zeros(nn), np.zeros(3 * nn), np.zeros(nn)
        _bcheck(_LIB.lbm_batch_fields(self._h, int(i), rho.ctypes.data, u.ctypes.data, c.ctypes.data), self._h)
        return rho.reshape(shape), u.reshape((3,) + shape), c.reshape(shape)

    def conversion_map(self, i):
        shape = self.shapes[i]
        out = np.zeros(int(np.prod(shape)))
        _bcheck(_LIB.lbm_batch_conversion_map(self._h, int(i), out.ctypes.data), self._h)
        return out.reshape(shape)

    def totals(self, i):
        t = lbm_totals_t()
        _bcheck(_LIB.lbm_batch_totals(self._h, int(i), ctypes.byref(t)), self._h)
        return {k: getattr(t, k) for k, _ in lbm_totals_t._fields_ if k != "reserved"}

    def info(self, i):
        inf = lbm_info()
        _bcheck(_LIB.lbm_batch_query(self._h, int(i), ctypes.byref(inf)), self._h)
        return {k: getattr(inf, k) for k, _ in lbm_info._fields_}
