"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, the ctypes structs match the C layouts, and parameter
validation returns status codes without touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jgb.h")


def _lib():
    from paper_1311_4120_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:jgb_status|const char\*)\s+(jgb_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["jgb_plan", "jgb_potential", "jgb_energy", "jgb_potential_backward", "jgb_destroy",
                     "jgb_last_error", "jgb_transform", "jgb_nodes", "jgb_plan_info", "jgb_timing_begin",
                     "jgb_timing_end"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(jgb_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(L.lib, n)


def test_struct_layouts_match_c(tmp_path):
    L = _lib()
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "jgb.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu\\n", sizeof(jgb_params), sizeof(jgb_info),'
                   ' offsetof(jgb_params, stream), offsetof(jgb_params, kmax), offsetof(jgb_info, workspace_bytes));'
                   'printf("%zu %zu %zu %zu\\n", offsetof(jgb_params, window), offsetof(jgb_info, window),'
                   ' offsetof(jgb_params, dipole_axis2), offsetof(jgb_params, alpha));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(L.Params)
    assert vals[1] == ctypes.sizeof(L.Info)
    assert vals[2] == L.Params.stream.offset
    assert vals[3] == L.Params.kmax.offset
    assert vals[4] == L.Info.workspace_bytes.offset
    assert vals[5] == L.Params.window.offset
    assert vals[6] == L.Info.window.offset
    assert vals[7] == L.Params.dipole_axis2.offset
    assert vals[8] == L.Params.alpha.offset


def _params(**kw):
    L = _lib()
    p = L.Params()
    p.struct_size = ctypes.sizeof(L.Params)
    p.dim = 3
    for i in range(3):
        p.n[i] = 16
        p.box[i] = 8.0
    p.kernel = L.COULOMB_3D
    p.dipole_axis[2] = 1.0
    p.lam = 1.0
    p.eps = 1e-10
    p.precision = L.FP64
    p.n_r, p.n_theta, p.n_phi = 8, 6, 12
    p.theta_rule = L.THETA_GL
    p.kmax = 0.0
    p.device = 0
    p.stream = None
    p.flags = 0
    for k, v in kw.items():
        if k in ("n", "box", "dipole_axis", "window", "dipole_axis2"):
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        else:
            setattr(p, k, v)
    return p


BAD = [
    ("struct_size", dict(struct_size=4), 1),
    ("dim", dict(dim=4), 1),
    ("odd n", dict(n=(15, 16, 16)), 1),
    ("small n", dict(n=(6, 16, 16)), 1),
    ("large n", dict(n=(1024, 16, 16)), 1),
    ("n with factor 7", dict(n=(14, 16, 16)), 2),
    ("box", dict(box=(8.0, -1.0, 8.0)), 1),
    ("kernel/dim", dict(kernel=1), 1),
    ("unknown kernel", dict(kernel=9), 1),
    ("dipole axis", dict(kernel=2, dipole_axis=(1.0, 1.0, 0.0)), 1),
    ("lambda", dict(lam=float("nan")), 1),
    ("eps small", dict(eps=1e-15), 1),
    ("eps large", dict(eps=0.5), 1),
    ("mixed eps", dict(precision=1, eps=1e-8), 1),
    ("precision", dict(precision=3), 1),
    ("n_r", dict(n_r=0), 1),
    ("n_theta", dict(n_theta=0), 1),
    ("odd n_phi", dict(n_phi=7), 1),
    ("theta rule", dict(theta_rule=5), 1),
    ("kmax too large", dict(kmax=100.0), 1),
    ("flags", dict(flags=64), 1),
    ("gaussian kernel below six digits", dict(flags=32, eps=1e-8), 2),
    ("radial rule too large", dict(flags=16, n_r=4096), 2),
    ("interp tiles in 2D", dict(flags=4, dim=2, kernel=1), 2),
    ("spread rings in 2D", dict(flags=8, dim=2, kernel=1), 2),
    ("window without split", dict(window=(1.0, 0.0)), 1),
    ("window nan", dict(flags=2, window=(float("nan"), 0.0)), 1),
    ("3D window[1]", dict(flags=2, window=(1.0, 2.0)), 1),
    ("3D negative a", dict(flags=2, window=(-1.0, 0.0)), 1),
    ("2D R0 >= R1", dict(flags=2, dim=2, kernel=1, window=(2.0, 1.0)), 1),
    ("2D R0 = 0", dict(flags=2, dim=2, kernel=1, window=(0.0, 1.0)), 1),
    ("split kmax too large", dict(flags=2, kmax=100.0), 1),
    ("dipole2d needs dim 2", dict(kernel=3), 1),
    ("dipole_axis2 not unit", dict(kernel=2, dipole_axis2=(0.5, 0.0, 0.0)), 1),
    ("dipole_axis2 nan", dict(kernel=2, dipole_axis2=(float("nan"), 0.0, 1.0)), 1),
    ("alpha nan", dict(alpha=float("nan")), 1),
    ("dipole2d axis not unit", dict(dim=2, kernel=3, dipole_axis=(0.6, 0.0, 0.0)), 1),
    ("poisson2d needs dim 2", dict(kernel=4), 1),
    # 33.5 M half-set nodes x 320-byte fp64 records: past the 32-bit table offsets
    ("node tables over 4 GiB", dict(n_r=512, n_theta=256, n_phi=512), 2),
    ("node tables over 4 GiB, mixed", dict(precision=1, eps=1e-5, n_r=1024, n_theta=512, n_phi=512), 2),
]


@pytest.mark.parametrize("name,kw,code", BAD, ids=[b[0] for b in BAD])
def test_invalid_parameters_return_status(name, kw, code):
    L = _lib()
    p = _params(**kw)
    h = ctypes.c_void_p()
    st = L.lib.jgb_plan(ctypes.byref(p), ctypes.byref(h))
    assert st == code, (st, L.lib.jgb_last_error())
    assert not h.value
    assert L.lib.jgb_last_error()


def test_null_arguments():
    L = _lib()
    h = ctypes.c_void_p()
    assert L.lib.jgb_plan(None, ctypes.byref(h)) == L.JGB_ERR_INVALID_ARG
    p = _params()
    assert L.lib.jgb_plan(ctypes.byref(p), None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_potential(None, None, None, None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_potential_noalloc(None, None, None, None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_energy(None, None, None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_potential_backward(None, None, None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_transform(None, None, None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_nodes(None, None, None, None) == L.JGB_ERR_INVALID_ARG
    info = L.Info()
    info.struct_size = ctypes.sizeof(L.Info)
    assert L.lib.jgb_plan_info(None, ctypes.byref(info)) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_timing_begin(None, 10) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_destroy(None) == L.JGB_OK


def test_valid_parameters_without_gpu_report_device_error():
    # on a host without a GPU a valid request fails cleanly with JGB_ERR_DEVICE
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib()
    for kw in (dict(), dict(flags=L.FLAG_SPLIT), dict(flags=L.FLAG_SPLIT, window=(0.7, 0.0)),
               dict(flags=L.FLAG_SPLIT, dim=2, kernel=L.COULOMB_2D, window=(0.3, 4.0)),
               dict(kernel=L.DIPOLE_3D, dipole_axis2=(1.0, 0.0, 0.0)),
               dict(dim=2, kernel=L.DIPOLE_2D, dipole_axis=(0.6, 0.0, 0.8), alpha=0.5)):
        p = _params(**kw)
        h = ctypes.c_void_p()
        assert L.lib.jgb_plan(ctypes.byref(p), ctypes.byref(h)) == L.JGB_ERR_DEVICE, kw
        assert not h.value


def test_package_refuses_to_run_without_library(tmp_path, monkeypatch):
    # the binding has no CPU fallback: a missing library is an ImportError
    import importlib.util
    L = _lib()
    spec = importlib.util.spec_from_file_location("jgb_lib_copy", L.__file__)
    mod = importlib.util.module_from_spec(spec)
    monkeypatch.setattr(os.path, "exists", lambda p: False if p.endswith("libjgb.so") else os.path.isfile(p))
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1311_4120_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def _gpe_params(**kw):
    L = _lib()
    g = L.GpeParams()
    g.struct_size = ctypes.sizeof(L.GpeParams)
    g.potential = _params()
    g.dt = 0.01
    g.beta = 1.0
    g.imaginary = 0
    for k, v in kw.items():
        if k == "trap":
            for i, x in enumerate(v):
                g.trap[i] = x
        else:
            setattr(g, k, v)
    return g


GPE_BAD = [
    ("struct_size", dict(struct_size=8)),
    ("dt zero", dict(dt=0.0)),
    ("dt nan", dict(dt=float("nan"))),
    ("beta inf", dict(beta=float("inf"))),
    ("imaginary flag", dict(imaginary=2)),
    ("trap nan", dict(trap=(1.0, float("nan"), 1.0))),
]


@pytest.mark.parametrize("name,kw", GPE_BAD, ids=[b[0] for b in GPE_BAD])
def test_gpe_invalid_parameters(name, kw):
    L = _lib()
    g = _gpe_params(**kw)
    h = ctypes.c_void_p()
    assert L.lib.jgb_gpe_create(ctypes.byref(g), ctypes.byref(h)) == L.JGB_ERR_INVALID_ARG
    assert not h.value
    assert L.lib.jgb_last_error()


def test_gpe_null_arguments_and_layout(tmp_path):
    L = _lib()
    h = ctypes.c_void_p()
    assert L.lib.jgb_gpe_create(None, ctypes.byref(h)) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_gpe_step(None, None, 1, 1) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_gpe_energy(None, None, None) == L.JGB_ERR_INVALID_ARG
    assert L.lib.jgb_gpe_destroy(None) == L.JGB_OK
    src = tmp_path / "g.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "jgb.h"\n'
                   'int main(){printf("%zu %zu %zu %zu\\n", sizeof(jgb_gpe_params), offsetof(jgb_gpe_params, V),'
                   ' offsetof(jgb_gpe_params, dt), offsetof(jgb_gpe_params, imaginary)); return 0;}\n')
    exe = tmp_path / "g"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(L.GpeParams), L.GpeParams.V.offset, L.GpeParams.dt.offset,
                    L.GpeParams.imaginary.offset]


def test_gpe_invalid_potential_is_reported():
    # the driver's own fields are valid, the potential's are not: the plan's error comes back
    L = _lib()
    g = _gpe_params()
    g.potential.dim = 5
    h = ctypes.c_void_p()
    assert L.lib.jgb_gpe_create(ctypes.byref(g), ctypes.byref(h)) == L.JGB_ERR_INVALID_ARG
    assert b"potential plan" in L.lib.jgb_last_error()


def test_noalloc_scratch_size_matches_header():
    L = _lib()
    m = re.search(r"#define JGB_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == L.NOALLOC_SCRATCH_BYTES


def test_flag_constants_match_the_header():
    """Every JGB_FLAG_* of include/jgb.h has the same value in the binding."""
    import paper_1311_4120_amd._lib as L
    flags = re.findall(r"#define JGB_FLAG_(\w+) (\d+)u", open(HEADER).read())
    assert len(flags) >= 7
    for name, val in flags:
        assert getattr(L, "FLAG_" + name) == int(val), name
