"""ctypes front end of the C oracle (test infrastructure only).

Arrays are numpy float64, populations laid out (q, nz, ny, nx) C-order, i.e.
f[a, z, y, x] == f[a*N + x + nx*(y + ny*z)] in the C code.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")


class Problem(C.Structure):
    _fields_ = [
        ("q", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("s", C.c_double * 26),
        ("face", C.c_int * 6),
        ("wall_u", (C.c_double * 3) * 6),
        ("F0", C.c_double * 3), ("FA", C.c_double * 3),
        ("FT", C.c_double),
        ("face_p0", C.c_double * 6), ("face_pA", C.c_double * 6),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        P = C.POINTER(Problem)
        L.orc_lattice.argtypes = [C.c_int, ip, dp, ip, dp, ip, dp]
        L.orc_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_macro_node.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_meq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_mforce.argtypes = [C.c_int, dp, dp, dp]
        L.orc_collide.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_init_eq.argtypes = [P, C.c_longlong, C.c_void_p, C.c_void_p,
                                  C.c_double, dp, dp]
        L.orc_run.argtypes = [P, C.c_longlong, C.c_longlong, dp]
        L.orc_macros.argtypes = [P, C.c_longlong, dp, dp, dp]
        L.orc_threads.argtypes = []
        _lib = L
    return _lib


def _chk(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed (rc=%d)" % (what, rc))


def lattice(q):
    """(c[q,3], w[q], opp[q], w0, T[q,q], N[q]) as the oracle holds them."""
    c = np.zeros(3 * q, np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, np.int32)
    w0 = np.zeros(1)
    T = np.zeros(q * q, np.int32)
    Nk = np.zeros(q)
    _chk(lib().orc_lattice(q, c, w, opp, w0, T, Nk), "lattice")
    return c.reshape(q, 3), w, opp, float(w0[0]), T.reshape(q, q), Nk


def feq(q, p, u):
    out = np.zeros(q)
    _chk(lib().orc_feq(q, float(p), np.asarray(u, np.float64), out), "feq")
    return out


def macro_node(q, f, F=(0.0, 0.0, 0.0)):
    p = np.zeros(1)
    u = np.zeros(3)
    _chk(lib().orc_macro_node(q, np.ascontiguousarray(f, np.float64),
                              np.asarray(F, np.float64), p, u), "macro_node")
    return float(p[0]), u


def meq(q, p, u):
    out = np.zeros(q)
    _chk(lib().orc_meq(q, float(p), np.asarray(u, np.float64), out), "meq")
    return out


def mforce(q, u, F):
    out = np.zeros(q)
    _chk(lib().orc_mforce(q, np.asarray(u, np.float64), np.asarray(F, np.float64), out),
         "mforce")
    return out


def collide(q, s, f, F=(0.0, 0.0, 0.0)):
    out = np.zeros(q)
    s26 = np.zeros(26)
    s26[:q] = s
    _chk(lib().orc_collide(q, s26, np.ascontiguousarray(f, np.float64),
                           np.asarray(F, np.float64), out), "collide")
    return out


def problem(q, nx, ny, nz, s, faces=("periodic",) * 6, wall_u=None,
            F0=(0.0, 0.0, 0.0), FA=(0.0, 0.0, 0.0), FT=0.0, face_p=None, face_pA=None):
    """faces: 6 entries 'periodic'/'wall'/'symmetry'/'velocity'/'pressure' in
    the order -x,+x,-y,+y,-z,+z; wall_u: dict face-name -> (ux,uy,uz) or a
    6x3 array (walls and velocity faces); face_p / face_pA: dict face-name ->
    pressure p0 / amplitude pA of a pressure face, p(t) = p0 + pA cos(2 pi t/FT)."""
    pr = Problem()
    pr.q, pr.nx, pr.ny, pr.nz = q, nx, ny, nz
    for k in range(q):
        pr.s[k] = float(s[k])
    for i, fk in enumerate(faces):
        pr.face[i] = {"periodic": 0, "wall": 1, "symmetry": 2, "velocity": 3, "pressure": 4,
                      "symmetry_node": 5, 0: 0, 1: 1, 2: 2, 3: 3, 4: 4, 5: 5}[fk]
    for name, v in (face_p or {}).items():
        pr.face_p0[FACES.index(name)] = float(v)
    for name, v in (face_pA or {}).items():
        pr.face_pA[FACES.index(name)] = float(v)
    if wall_u is not None:
        if isinstance(wall_u, dict):
            for name, v in wall_u.items():
                i = FACES.index(name)
                for d in range(3):
                    pr.wall_u[i][d] = float(v[d])
        else:
            wu = np.asarray(wall_u, np.float64).reshape(6, 3)
            for i in range(6):
                for d in range(3):
                    pr.wall_u[i][d] = wu[i, d]
    for d in range(3):
        pr.F0[d] = float(F0[d])
        pr.FA[d] = float(FA[d])
    pr.FT = float(FT)
    return pr


def init_eq(pr, t=0, p=None, u=None, p0=0.0, u0=(0.0, 0.0, 0.0)):
    q, nx, ny, nz = pr.q, pr.nx, pr.ny, pr.nz
    f = np.zeros((q, nz, ny, nx))
    pp = None if p is None else np.ascontiguousarray(p, np.float64)
    uu = None if u is None else np.ascontiguousarray(u, np.float64)
    _chk(lib().orc_init_eq(C.byref(pr), int(t),
                           None if pp is None else pp.ctypes.data,
                           None if uu is None else uu.ctypes.data,
                           float(p0), np.asarray(u0, np.float64), f), "init_eq")
    return f


def run(pr, f, t0, nsteps):
    """Advance a copy of f (q,nz,ny,nx) from time level t0 by nsteps."""
    g = np.ascontiguousarray(f, np.float64).copy()
    _chk(lib().orc_run(C.byref(pr), int(t0), int(nsteps), g), "run")
    return g


def macros(pr, f, t):
    """(p[nz,ny,nx], u[3,nz,ny,nx]) at time level t."""
    nx, ny, nz = pr.nx, pr.ny, pr.nz
    p = np.zeros((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    _chk(lib().orc_macros(C.byref(pr), int(t), np.ascontiguousarray(f, np.float64), p, u),
         "macros")
    return p, u


def threads():
    return int(lib().orc_threads())
