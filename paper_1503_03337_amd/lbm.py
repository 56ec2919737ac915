"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the lattice Boltzmann path runs in the HIP kernels of the
library.  PyTorch is used for device memory (the population buffer of a
lattice is a torch tensor when torch sees a GPU) and for streams.  There is
no fallback: if the library is missing, loading raises.

Array conventions: populations f[a, z, y, x] (q, nz, ny, nx) float64,
pressure p[z, y, x], velocity u[d, z, y, x] (3, nz, ny, nx), matching the
library's [q][N] / [3][N] layouts with n = x + nx*(y + ny*z).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIB_PATH selects another build of the same ABI (for A/B measurements
# of kernel variants); by default the in-tree build.
LIB_PATH = os.environ.get("LBM_LIB_PATH") or os.path.join(HERE, "liblbm.so")

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2}
ROUNDING = {"stochastic": 0, "nearest": 1}
COLLISION = {"mrt": 0, "bgk": 1}
PATTERN = {"ab": 0, "aa": 1}
FACE_KIND = {"periodic": 0, "wall": 1, "symmetry": 2, "velocity": 3, "pressure": 4,
             "symmetry_node": 5}
OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5
NOALLOC_MAX_NODES = 262144  # LBM_NOALLOC_MAX_NODES
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_ENONFINITE", -5: "LBM_ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Spec(C.Structure):
    _fields_ = [
        ("face", C.c_int * 6),
        ("wall_u", (C.c_double * 3) * 6),
        ("F0", C.c_double * 3),
        ("FA", C.c_double * 3),
        ("FT", C.c_double),
        ("p0", C.c_double),
        ("u0", C.c_double * 3),
        ("storage", C.c_int),
        ("pattern", C.c_int),
        ("f16_scale_log2", C.c_int),
        ("f16_rounding", C.c_int),
        ("collision", C.c_int),
        ("monitor_every", C.c_int),
        ("stream", C.c_void_p),
        ("dev_buf", C.c_void_p),
        ("dev_buf_bytes", C.c_size_t),
        ("face_p", C.c_double * 6),
        ("face_pA", C.c_double * 6),
        ("graphs", C.c_int),
    ]


class Info(C.Structure):
    _fields_ = [
        ("q", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("storage", C.c_int), ("pattern", C.c_int),
        ("t", C.c_longlong),
        ("nodes", C.c_size_t),
        ("population_bytes", C.c_size_t),
        ("footprint_bytes", C.c_size_t),
        ("bytes_per_value", C.c_int),
        ("graphs", C.c_int),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # torch ships its own HIP runtime under the same soname; load it first
        # so that liblbm.so binds to that one instead of a second copy (two
        # HIP runtimes in one process do not share the device, streams or
        # pointers).
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - torch is part of the image
            pass
        L = C.CDLL(LIB_PATH)
        vp, i, ll, d, sz = C.c_void_p, C.c_int, C.c_longlong, C.c_double, C.c_size_t
        dp = C.POINTER(C.c_double)
        sig = {
            "lbm_spec_default": (None, [C.POINTER(Spec)]),
            "lbm_footprint_bytes": (sz, [i, i, i, i, C.POINTER(Spec)]),
            "lbm_create": (i, [C.POINTER(vp), i, i, i, i, dp, C.POINTER(Spec)]),
            "lbm_step": (i, [vp, ll]),
            "lbm_macros": (i, [vp, dp, dp]),
            "lbm_macros_device": (i, [vp, vp, vp]),
            "lbm_macros_noalloc": (i, [vp, ll, ll, dp, dp]),
            "lbm_residual": (i, [vp, dp]),
            "lbm_residual_change": (i, [vp, dp, C.POINTER(ll)]),
            "lbm_poll": (i, [vp]),
            "lbm_mass": (i, [vp, dp]),
            "lbm_monitor": (i, [vp]),
            "lbm_get_f": (i, [vp, dp]),
            "lbm_set_f": (i, [vp, dp]),
            "lbm_init_fields": (i, [vp, dp, dp]),
            "lbm_time": (ll, [vp]),
            "lbm_set_time": (i, [vp, ll]),
            "lbm_info": (i, [vp, C.POINTER(Info)]),
            "lbm_sync": (i, [vp]),
            "lbm_last_error": (C.c_char_p, [vp]),
            "lbm_status_string": (C.c_char_p, [i]),
            "lbm_destroy": (i, [vp]),
            "lbm_batch_create": (i, [C.POINTER(vp), vp]),
            "lbm_batch_add": (i, [vp, vp, ll]),
            "lbm_batch_remove": (i, [vp, vp]),
            "lbm_batch_set_tile": (i, [vp, vp, i, i]),
            "lbm_batch_step": (i, [vp, ll]),
            "lbm_batch_monitor": (i, [vp]),
            "lbm_batch_remaining": (ll, [vp, vp]),
            "lbm_batch_size": (i, [vp]),
            "lbm_batch_last_error": (C.c_char_p, [vp]),
            "lbm_batch_destroy": (i, [vp]),
            "lbm_copy_probe": (i, [vp, vp, sz, i, vp]),
            "lbm_pattern_probe": (i, [vp, i, i, i, i, i, ll, i, i, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_spec(faces=("wall",) * 6, wall_u=None, F0=(0, 0, 0), FA=(0, 0, 0), FT=0.0, p0=0.0,
              u0=(0, 0, 0), storage="f32", pattern="aa", f16_scale_log2=12,
              f16_rounding="stochastic", collision="mrt", monitor_every=0, stream=None,
              face_p=None, face_pA=None, graphs=True):
    """face_p / face_pA: {face name: value} pressures of pressure faces,
    p(t) = face_p + face_pA cos(2 pi t / FT)."""
    sp = Spec()
    lib().lbm_spec_default(C.byref(sp))
    for k, fk in enumerate(faces):
        sp.face[k] = FACE_KIND[fk] if isinstance(fk, str) else int(fk)
    if wall_u is not None:
        if isinstance(wall_u, dict):
            for name, v in wall_u.items():
                for dd in range(3):
                    sp.wall_u[FACES.index(name)][dd] = float(v[dd])
        else:
            w = np.asarray(wall_u, np.float64).reshape(6, 3)
            for k in range(6):
                for dd in range(3):
                    sp.wall_u[k][dd] = float(w[k, dd])
    for dd in range(3):
        sp.F0[dd] = float(F0[dd])
        sp.FA[dd] = float(FA[dd])
        sp.u0[dd] = float(u0[dd])
    sp.FT = float(FT)
    sp.p0 = float(p0)
    sp.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    sp.pattern = PATTERN[pattern] if isinstance(pattern, str) else int(pattern)
    sp.f16_scale_log2 = int(f16_scale_log2)
    sp.f16_rounding = ROUNDING[f16_rounding] if isinstance(f16_rounding, str) else int(f16_rounding)
    sp.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    sp.monitor_every = int(monitor_every)
    sp.stream = stream
    sp.graphs = 1 if graphs else 0
    for name, v in (face_p or {}).items():
        sp.face_p[FACES.index(name)] = float(v)
    for name, v in (face_pA or {}).items():
        sp.face_pA[FACES.index(name)] = float(v)
    return sp


def footprint_bytes(model, nx, ny, nz, **spec_kw):
    sp = make_spec(**spec_kw)
    return int(lib().lbm_footprint_bytes(int(model), int(nx), int(ny), int(nz), C.byref(sp)))


def _torch_stream_and_buffer(nbytes, use_torch):
    """(stream handle, buffer tensor or None) from torch, if it sees a GPU."""
    if not use_torch:
        return None, None
    try:
        import torch
    except ImportError:  # pragma: no cover - torch is part of the image
        return None, None
    if not torch.cuda.is_available():
        return None, None
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    return torch.cuda.current_stream().cuda_stream, buf


class Lattice:
    """One lattice (a context of the C library)."""

    def __init__(self, model, nx, ny, nz, s_vec, use_torch=True, stream=None, **spec_kw):
        L = lib()
        self.q, self.nx, self.ny, self.nz = int(model), int(nx), int(ny), int(nz)
        s = np.ascontiguousarray(s_vec, np.float64)
        if s.shape != (self.q,):
            raise ValueError("s_vec must hold q = %d rates" % self.q)
        sp = make_spec(**spec_kw)
        need = L.lbm_footprint_bytes(self.q, self.nx, self.ny, self.nz, C.byref(sp))
        if need == 0:
            raise LbmError(-1, "invalid lattice description")
        tstream, self._buf = _torch_stream_and_buffer(need, use_torch)
        self._buf_stream = tstream  # stream torch allocated the buffer on
        if stream is None:
            stream = tstream
        sp.stream = stream
        if self._buf is not None:
            sp.dev_buf = self._buf.data_ptr()
            sp.dev_buf_bytes = need
        self.stream = stream
        self.spec = sp
        h = C.c_void_p()
        rc = L.lbm_create(C.byref(h), self.q, self.nx, self.ny, self.nz, _dptr(s), C.byref(sp))
        if rc != 0:
            raise LbmError(rc, "lbm_create: " + L.lbm_last_error(None).decode())
        self.h = h
        self.s_vec = s

    # -- helpers
    def _chk(self, rc, what):
        if rc != 0:
            raise LbmError(rc, "%s: %s" % (what, lib().lbm_last_error(self.h).decode()))

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def time(self):
        return int(lib().lbm_time(self.h))

    def set_time(self, t):
        self._chk(lib().lbm_set_time(self.h, int(t)), "lbm_set_time")

    def info(self):
        inf = Info()
        self._chk(lib().lbm_info(self.h, C.byref(inf)), "lbm_info")
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    # -- the ABI
    def step(self, n=1):
        self._chk(lib().lbm_step(self.h, int(n)), "lbm_step")

    def sync(self):
        self._chk(lib().lbm_sync(self.h), "lbm_sync")

    def macros(self):
        p = np.empty((self.nz, self.ny, self.nx))
        u = np.empty((3, self.nz, self.ny, self.nx))
        self._chk(lib().lbm_macros(self.h, _dptr(p), _dptr(u)), "lbm_macros")
        return p, u

    def macros_noalloc(self, n0, count):
        """(p[count], u[3, count]) of nodes [n0, n0 + count) through
        lbm_macros_noalloc (no allocation; count <= NOALLOC_MAX_NODES)."""
        m = max(int(count), 0)  # the library rejects a negative count itself
        p = np.empty(m)
        u = np.empty((3, m))
        self._chk(lib().lbm_macros_noalloc(self.h, int(n0), int(count), _dptr(p), _dptr(u)),
                  "lbm_macros_noalloc")
        return p, u

    def macros_device(self, p_ptr, u_ptr):
        self._chk(lib().lbm_macros_device(self.h, p_ptr, u_ptr), "lbm_macros_device")

    def monitor(self):
        self._chk(lib().lbm_monitor(self.h), "lbm_monitor")

    def residual(self):
        r = C.c_double()
        self._chk(lib().lbm_residual(self.h, C.byref(r)), "lbm_residual")
        return r.value

    def residual_change(self):
        """(R_L, L): the change of u over the monitor's lag L in the norm of
        the paper's steady-state criteria (not divided by L)."""
        r = C.c_double()
        lag = C.c_longlong()
        self._chk(lib().lbm_residual_change(self.h, C.byref(r), C.byref(lag)),
                  "lbm_residual_change")
        return r.value, int(lag.value)

    def poll(self):
        """Raise LbmError (LBM_ENONFINITE) if a completed monitor run has seen
        a non-finite value; never waits for the device."""
        self._chk(lib().lbm_poll(self.h), "lbm_poll")

    def healthy(self):
        """False once a completed monitor run has seen a non-finite value."""
        return lib().lbm_poll(self.h) != ENONFINITE

    def mass(self):
        m = C.c_double()
        self._chk(lib().lbm_mass(self.h, C.byref(m)), "lbm_mass")
        return m.value

    def get_f(self):
        f = np.empty((self.q, self.nz, self.ny, self.nx))
        self._chk(lib().lbm_get_f(self.h, _dptr(f)), "lbm_get_f")
        return f

    def set_f(self, f):
        f = np.ascontiguousarray(f, np.float64)
        if f.shape != (self.q, self.nz, self.ny, self.nx):
            raise ValueError("f must have shape (q, nz, ny, nx)")
        self._chk(lib().lbm_set_f(self.h, _dptr(f)), "lbm_set_f")

    def init_fields(self, p=None, u=None):
        pp = None if p is None else np.ascontiguousarray(p, np.float64)
        uu = None if u is None else np.ascontiguousarray(u, np.float64)
        if pp is not None and pp.size != self.N:
            raise ValueError("p must hold N values")
        if uu is not None and uu.size != 3 * self.N:
            raise ValueError("u must hold 3N values")
        self._chk(lib().lbm_init_fields(self.h, None if pp is None else _dptr(pp),
                                        None if uu is None else _dptr(uu)), "lbm_init_fields")

    def close(self):
        """Destroy the context.  The population buffer (a torch tensor) is
        released to torch's caching allocator, which orders its reuse after
        the work already queued on the stream it was allocated on; when the
        lattice ran on another stream, that stream is drained first."""
        if getattr(self, "h", None):
            if self._buf is not None and self.stream != self._buf_stream:
                lib().lbm_sync(self.h)
            lib().lbm_destroy(self.h)
            self.h = None
            self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many lattices advanced together, one kernel launch per time step."""

    def __init__(self, stream=None):
        h = C.c_void_p()
        rc = lib().lbm_batch_create(C.byref(h), stream)
        if rc != 0:
            raise LbmError(rc, "lbm_batch_create failed")
        self.h = h
        self.members = []

    def _chk(self, rc, what):
        if rc != 0:
            raise LbmError(rc, "%s: %s" % (what, lib().lbm_batch_last_error(self.h).decode()))

    def add(self, lat, budget):
        self._chk(lib().lbm_batch_add(self.h, lat.h, int(budget)), "lbm_batch_add")
        self.members.append(lat)

    def remove(self, lat):
        # a closed lattice already left the batch when it was destroyed
        if lat.h is not None:
            self._chk(lib().lbm_batch_remove(self.h, lat.h), "lbm_batch_remove")
        self.members.remove(lat)

    def set_tile(self, lat, tx, ty):
        self._chk(lib().lbm_batch_set_tile(self.h, lat.h, int(tx), int(ty)), "lbm_batch_set_tile")

    def step(self, n):
        self._chk(lib().lbm_batch_step(self.h, int(n)), "lbm_batch_step")

    def monitor(self):
        self._chk(lib().lbm_batch_monitor(self.h), "lbm_batch_monitor")

    def remaining(self, lat):
        return int(lib().lbm_batch_remaining(self.h, lat.h))

    def __len__(self):
        return int(lib().lbm_batch_size(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_batch_destroy(self.h)
            self.h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_probe(dst_ptr, src_ptr, nbytes, reps=1, stream=None):
    rc = lib().lbm_copy_probe(dst_ptr, src_ptr, int(nbytes), int(reps), stream)
    if rc != 0:
        raise LbmError(rc, "lbm_copy_probe failed")


def pattern_probe(buf_ptr, q, elem_bytes, shape, stride, odd=False, reps=1, stream=None):
    nx, ny, nz = shape
    rc = lib().lbm_pattern_probe(buf_ptr, int(q), int(elem_bytes), int(nx), int(ny), int(nz),
                                 int(stride), int(bool(odd)), int(reps), stream)
    if rc != 0:
        raise LbmError(rc, "lbm_pattern_probe failed")
