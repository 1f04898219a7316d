"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid configurations before touching any device."""
import ctypes
import math
import os
import re

import pytest

from paper_2102_08756_amd import sbim as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbim_[a-z_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = B.load_library()
    names = declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def _cfg(**kw):
    c = B._Config()
    c.n1, c.n3, c.dx1, c.dx3, c.dt = 8, 8, 1.0, 1.0, 0.2
    c.nplanes = 1
    c.plane[0] = B._Plane(1, 1.0, 1.0, math.sqrt(3.0))
    c.window_cap, c.window_mode, c.eta_w = 10, 0, 1.0
    c.precision, c.input_kind, c.stream = 0, 0, None
    for k, v in kw.items():
        if k.startswith("plane0_"):
            p = c.plane[0]
            setattr(p, k[7:], v)
            c.plane[0] = p
        else:
            setattr(c, k, v)
    return c


@pytest.mark.parametrize("bad, msg", [
    (dict(n1=12), "power of two"), (dict(n3=2), "power of two"), (dict(n1=8192), "power of two"),
    (dict(dt=0.0), "dt"), (dict(dx1=-1.0), "dx1"), (dict(dt=float("nan")), "dt"),
    (dict(nplanes=3), "nplanes"), (dict(nplanes=0), "nplanes"),
    (dict(plane0_side=0), "side"), (dict(plane0_mu=0.0), "mu"),
    (dict(plane0_cp=1.1), "cp="), (dict(window_cap=0), "window_cap"),
    (dict(window_mode=7), "window_mode"), (dict(window_mode=1, eta_w=0.0), "eta_w"),
    (dict(precision=5), "precision"), (dict(input_kind=3), "input_kind"),
])
def test_invalid_configs_rejected_on_host(bad, msg):
    lib = B.load_library()
    c = _cfg(**bad)
    h = ctypes.c_void_p(123)
    rc = lib.sbim_init(ctypes.byref(c), ctypes.byref(h))
    assert rc == B.SBIM_E_INVALID
    assert h.value is None
    assert msg in lib.sbim_last_error(None).decode()


def test_null_arguments_rejected():
    lib = B.load_library()
    assert lib.sbim_init(None, None) == B.SBIM_E_INVALID
    assert lib.sbim_push_displacement(None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_tractions(None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_backward(None, None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_destroy(None) == B.SBIM_OK
    assert lib.sbim_state_bytes(None) == -1
    assert lib.sbim_fault_create(None, None, None) == B.SBIM_E_INVALID
    f = ctypes.c_void_p(123)
    assert lib.sbim_fault_create(None, None, ctypes.byref(f)) == B.SBIM_E_INVALID
    assert f.value is None
    assert lib.sbim_fault_step(None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_fault_read(None, 0, None) == B.SBIM_E_INVALID
    assert lib.sbim_fault_reset(None) == B.SBIM_E_INVALID
    assert lib.sbim_fault_destroy(None) == B.SBIM_OK
    assert lib.sbim_strip_create(None, None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_strip_step(None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_strip_read(None, 0, None) == B.SBIM_E_INVALID
    assert lib.sbim_strip_reset(None) == B.SBIM_E_INVALID
    assert lib.sbim_strip_destroy(None) == B.SBIM_OK
    assert lib.sbim_set_dt(None, 0.1) == B.SBIM_E_INVALID
    assert lib.sbim_count_nonfinite(None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_count_nonfinite_noalloc(None, None, None) == B.SBIM_E_INVALID
    assert lib.sbim_traction_spectrum(None, None) == B.SBIM_E_INVALID


STRUCTS = {"sbim_plane": B._Plane, "sbim_config": B._Config, "sbim_info": B._Info,
           "sbim_fault_params": B._FaultParams, "sbim_strip_config": B._StripConfig}


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets that a C
    compiler gives the header's structs (a program built with gcc prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    body = []
    for cname, cls in STRUCTS.items():
        body.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            body.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"sbim.h\"\nint main(void) {\n"
                   + "\n".join(body) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                          text=True).stdout.splitlines())
    for cname, cls in STRUCTS.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
