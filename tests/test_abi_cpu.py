"""CPU-side checks of the C ABI: the built library loads and exports every
function include/lbm.h declares; the calls that touch no device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for core in ("lbm_create", "lbm_step", "lbm_macros", "lbm_residual", "lbm_mass",
                 "lbm_get_f", "lbm_set_f", "lbm_destroy", "lbm_batch_step"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1503_03337_amd import lbm
    L = lbm.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    # and the binding wraps each of them
    src = open(os.path.join(ROOT, "paper_1503_03337_amd", "lbm.py")).read()
    for name in declared_functions():
        assert '"%s"' % name in src, name


def test_footprint_without_device():
    """q arrays of N values (N rounded up to 64, plus a fixed pad of at most
    4096 values), one copy for AA, two for AB; the monitor adds 3N values."""
    from paper_1503_03337_amd import lbm

    def ok(got, q, N, b, copies):
        lo = copies * q * N * b
        return lo <= got <= copies * (q * (N + 64 + 4096) * b + 256)

    n = 128
    N = n ** 3
    assert ok(lbm.footprint_bytes(18, n, n, n, storage="f32", pattern="aa"), 18, N, 4, 1)
    assert ok(lbm.footprint_bytes(18, n, n, n, storage="f32", pattern="ab"), 18, N, 4, 2)
    assert ok(lbm.footprint_bytes(14, n, n, n, storage="f16dev", pattern="aa"), 14, N, 2, 1)
    assert ok(lbm.footprint_bytes(14, 16, 16, 32, storage="f64", pattern="ab"), 14, 8192, 8, 2)
    aa = lbm.footprint_bytes(18, n, n, n, storage="f32", pattern="aa")
    with_mon = lbm.footprint_bytes(18, n, n, n, storage="f32", pattern="aa", monitor_every=10)
    assert with_mon >= aa + 3 * N * 4


@pytest.mark.parametrize("bad", [
    dict(model=15), dict(nx=0), dict(faces=("periodic", "wall") + ("wall",) * 4),
    dict(wall_u={"+z": (0.3, 0, 0)}), dict(storage=7), dict(pattern=5),
    dict(storage="f16dev", f16_scale_log2=30), dict(monitor_every=-1),
    dict(faces=("periodic", "symmetry") + ("wall",) * 4), dict(faces=(6,) + ("wall",) * 5),
    dict(faces=("wall",) * 5 + (-1,)),
    dict(nx=2, faces=("pressure", "pressure") + ("velocity",) * 4),
    dict(faces=("pressure", "wall") + ("wall",) * 4, face_p={"-x": float("nan")}),
    dict(u0=(0.0, float("nan"), 0.0)), dict(FT=float("nan")), dict(FT=float("inf")),
    dict(p0=float("inf")), dict(F0=(float("nan"), 0.0, 0.0)),
])
def test_footprint_rejects_invalid(bad):
    from paper_1503_03337_amd import lbm
    args = dict(model=18, nx=8, ny=8, nz=8)
    args.update({k: v for k, v in bad.items() if k in args})
    kw = {k: v for k, v in bad.items() if k not in ("model", "nx", "ny", "nz")}
    assert lbm.footprint_bytes(args["model"], args["nx"], args["ny"], args["nz"], **kw) == 0


def test_status_strings():
    from paper_1503_03337_amd import lbm
    L = lbm.lib()
    assert L.lbm_status_string(0) == b"ok"
    assert L.lbm_status_string(-4) == b"non-finite value"


def test_create_rejects_bad_rates_without_device():
    """Validation happens before any device call."""
    import numpy as np
    from paper_1503_03337_amd import lbm
    L = lbm.lib()
    sp = lbm.make_spec()
    h = C.c_void_p()
    s = np.full(18, 2.0)
    assert L.lbm_create(C.byref(h), 18, 8, 8, 8, s.ctypes.data_as(C.POINTER(C.c_double)),
                        C.byref(sp)) == -1
    s = np.full(18, 1.0)
    assert L.lbm_create(C.byref(h), 16, 8, 8, 8, s.ctypes.data_as(C.POINTER(C.c_double)),
                        C.byref(sp)) == -1


def test_params_match_paper_rates():
    from paper_1503_03337_amd import params
    s = params.s_vec(14, nu=0.1)
    assert s[1] == 1.19 and s[3] == 1.2 and s[13] == 0.98 and s[0] == 1.0
    assert abs(s[8] - 1.25) < 1e-15
    from oracle import analytic
    assert abs(params.DUCT_UMAX_COEFF - analytic.duct_steady_umax_coeff()) < 1e-14


def test_serving_ducts_tie_odd_rates_to_viscosity():
    """Duct requests relax q and t at s_o with (1/s_nu - 1/2)(1/s_o - 1/2)
    = 3/16, keeping the paper's even rates; cavities keep the paper's set."""
    from paper_1503_03337_amd import params, serve
    for q in (14, 18):
        for edge in (32, 100, 160):
            s, _ = serve.request_setup({"q": q, "edge": edge, "kind": "duct"})
            sn = params.s_nu(serve.duct_nu(edge))
            odd = [3, 5, 7] + ([13] if q == 14 else [15, 16, 17])
            for k in odd:
                assert abs((1 / sn - 0.5) * (1 / s[k] - 0.5) - 3 / 16) < 1e-14
            assert s[1] == params.S_E and abs(s[8] - sn) < 1e-15
            if q == 18:
                assert s[9] == params.S_PI
        s, _ = serve.request_setup({"q": q, "edge": 64, "kind": "cavity"})
        assert s[3] == params.S_Q


def test_bgk_needs_equal_rates_without_device():
    import numpy as np
    from paper_1503_03337_amd import lbm
    L = lbm.lib()
    sp = lbm.make_spec(collision="bgk")
    h = C.c_void_p()
    s = np.full(18, 1.2)
    s[4] = 1.0
    assert L.lbm_create(C.byref(h), 18, 8, 8, 8, s.ctypes.data_as(C.POINTER(C.c_double)),
                        C.byref(sp)) == -1
    assert b"equal" in L.lbm_last_error(None)


def test_footprint_accepts_symmetry_faces():
    from paper_1503_03337_amd import lbm
    for faces in (("wall",) * 5 + ("symmetry",),
                  ("symmetry", "symmetry", "periodic", "periodic", "wall", "symmetry")):
        assert lbm.footprint_bytes(18, 8, 8, 8, faces=faces) > 0


def test_footprint_holds_the_boundary_node_list():
    """Velocity / pressure faces add the list of their nodes (int32) to the
    footprint: 17 x 9 x 9 duct, every face of that kind -> all nodes but the
    15 x 7 x 7 inner box."""
    from paper_1503_03337_amd import lbm
    faces = ("pressure", "pressure") + ("velocity",) * 4
    walls = lbm.footprint_bytes(14, 17, 9, 9, faces=("wall",) * 6, storage="f64")
    nee = lbm.footprint_bytes(14, 17, 9, 9, faces=faces, storage="f64")
    count = 17 * 9 * 9 - 15 * 7 * 7
    assert nee - walls == (4 * count + 255) // 256 * 256


def test_plain_c_program_links_and_validates():
    """tests/c_abi/lid_cavity.c uses nothing but include/lbm.h and
    liblbm.so (no Python, no torch); its validation-only mode makes no
    device call."""
    import os
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "lid_cavity")
    assert os.path.exists(exe), "build it with __graft_entry__.build()"
    out = subprocess.run([exe, "--check-only"], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert "validation ok" in out.stdout


def test_duct_error_norms_on_constructed_fields():
    """serve.duct_errors on fields with known errors: the exact series gives
    0, a uniform relative error e in u_x gives GRE_u = e and a max error of
    e * max|u| / u_max, a cross-flow v adds to GRE_u only."""
    import numpy as np
    from oracle import analytic
    from paper_1503_03337_amd import params, serve
    L = 12
    a = L / 2.0
    nu = serve.duct_nu(L)
    g = serve.DUCT_UMAX * nu / (params.DUCT_UMAX_COEFF * a * a)
    y = np.arange(L) + 0.5 - a
    Y, Z = np.meshgrid(y, y, indexing="xy")

    def series(Yv, Zv, av, gv, nuv):
        return analytic.duct_steady(Yv, Zv, av, av, gv, nuv)

    ua = series(Y, Z, a, g, nu)
    u = np.zeros((3, L, L, L))
    u[0] = ua[:, :, None]
    rec = {"edge": L, "u": u}
    assert serve.duct_errors(rec, series) == (0.0, 0.0)
    eps = 1e-3
    u[0] *= 1.0 + eps
    emax, gre = serve.duct_errors(rec, series)
    assert abs(gre - eps) < 1e-12
    assert abs(emax - eps * np.max(ua) / serve.DUCT_UMAX) < 1e-12
    u[0] = ua[:, :, None]
    u[1] = 0.5e-3 * np.max(ua)
    emax, gre = serve.duct_errors(rec, series)
    assert emax == 0.0
    expect = 0.5e-3 * np.max(ua) * np.sqrt(L ** 3 / (L * np.sum(ua ** 2)))
    assert abs(gre - expect) < 1e-12 * max(1.0, expect)
