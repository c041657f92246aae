"""CPU-only checks of the C ABI: the HIP library loads, exports every entry
point that include/epic.h declares, and its host-side logic (validation,
workspace sizing, error strings) behaves as documented.  No device call."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epic.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1501_02565_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libepic.so is not built (run __graft_entry__.build())")
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(epic_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    from paper_1501_02565_amd import _lib
    assert set(declared_functions()) == set(_lib.SYMBOLS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


P = ctypes.c_void_p(0x1000)   # never dereferenced by validation


def test_validate(lib):
    ok = lib.epic_validate(P, 10, 20, P, 5, 3, 1.0, 1, P)
    assert ok == 0
    bad = [
        (None, 10, 20, P, 5, 3, 1.0, 1, P),
        (P, 10, 20, None, 5, 3, 1.0, 1, P),
        (P, 10, 20, P, 5, 3, 1.0, 1, None),
        (P, 0, 20, P, 5, 3, 1.0, 1, P),
        (P, 10, 0, P, 5, 3, 1.0, 1, P),
        (P, 10, 20, P, 0, 3, 1.0, 1, P),
        (P, 10, 20, P, 5, 0, 1.0, 1, P),
        (P, 10, 20, P, 5, 257, 1.0, 1, P),
        (P, 10, 20, P, 5, 3, -0.5, 1, P),
        (P, 10, 20, P, 5, 3, float("nan"), 1, P),
        (P, 10, 20, P, 5, 3, float("inf"), 1, P),
        (P, 10, 20, P, 5, 3, 1.0, 2, P),
        (P, 65536, 32768, P, 5, 3, 1.0, 1, P),
    ]
    for args in bad:
        assert lib.epic_validate(*args) == -1, args


def test_interp_rejects_before_touching_the_device(lib):
    # invalid arguments are rejected on the host, before the context is used
    assert lib.epic_interp(None, P, 10, 20, P, 5, 3, -1.0, 1, P, None) == -1
    assert lib.epic_interp(None, P, 10, 20, P, 5, 3, 1.0, 1, P, None) == -1  # no context
    assert lib.epic_interp_batch(None, None, 1, None) == -1
    from paper_1501_02565_amd import _lib
    st = _lib.Stats()
    assert lib.epic_get_stats(None, 0, ctypes.byref(st)) == -1


def test_workspace_bytes(lib):
    f = lib.epic_workspace_bytes
    small = f(96, 128, 300, 32, 1, 0)
    big = f(436, 1024, 8000, 100, 1, 0)
    assert 0 < small < big
    assert f(436, 1024, 16000, 100, 1, 0) > big
    assert f(0, 10, 5, 3, 1, 0) == 0
    assert f(10, 10, 5, 0, 1, 0) == 0
    assert f(10, 10, 5, 3, 7, 0) == 0
    # 8 B/px transform state dominates the image-size term
    assert f(872, 1024, 8000, 100, 1, 0) - big >= 8 * 436 * 1024


def test_strerror(lib):
    for code in range(-8, 1):
        s = lib.epic_strerror(code).decode()
        assert s and s != "unknown status"
    assert lib.epic_strerror(42).decode() == "unknown status"


def _struct_fields(name):
    """Field names of `typedef struct ... { ... } name;` in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \w*\s*\{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            names += [v.strip().lstrip("*") for v in decl.split(None, 1)[1].replace("*", " ").split(",")]
    return [n.split()[-1] for n in names]


def test_binding_structs_follow_the_header():
    from paper_1501_02565_amd import _lib
    for cname, cls in (("epic_options", _lib.Options), ("epic_stats", _lib.Stats),
                       ("epic_request", _lib.Request), ("epic_image", _lib.Image),
                       ("epic_refine_params", _lib.RefineParams)):
        assert _struct_fields(cname) == [f for f, _ in cls._fields_], cname


def test_status_codes_follow_the_header():
    from paper_1501_02565_amd import _lib
    text = open(HEADER).read()
    for name, value in re.findall(r"EPIC_(OK|ERR_[A-Z_]+)\s*=\s*(-?\d+)", text):
        assert getattr(_lib, name) == int(value), name


def test_binding_loads_one_hip_runtime():
    """Loading the library first (before any torch import) must still leave
    a single HIP runtime in the process: the one torch uses."""
    import ast
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1501_02565_amd import _lib\n"
            "_lib.load()\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1501_02565_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()


def test_image_cost_rejects_bad_arguments(lib):
    from paper_1501_02565_amd import _lib
    good = _lib.Image(0x1000, 10, 20, 3, 0x2000)
    arr = (_lib.Image * 1)(good)
    bad_eps = [0.0, -1.0, float("nan"), float("inf")]
    for e in bad_eps:
        assert lib.epic_image_cost(arr, 1, e, None) == -1
    for fields in [dict(image=None), dict(cost=None), dict(H=0), dict(W=0), dict(channels=0),
                   dict(channels=5), dict(image=0x1002), dict(H=65536, W=32768)]:
        d = dict(image=0x1000, H=10, W=20, channels=3, cost=0x2000)
        d.update(fields)
        a = (_lib.Image * 1)(_lib.Image(d["image"], d["H"], d["W"], d["channels"], d["cost"]))
        assert lib.epic_image_cost(a, 1, 1e-3, None) == -1, fields
    assert lib.epic_image_cost(arr, 0, 1e-3, None) == -1
    assert lib.epic_interp_image(None, P, 10, 20, 3, 1e-3, P, 5, 3, 1.0, 1, P, None) == -1


def test_refine_defaults_and_bytes(lib):
    """The library's refinement defaults are the paper's (kappa 5, 5 outer
    iterations of 30 sweeps) and the oracle's; the scratch size is 104 + 4 C
    bytes per pixel plus alignment; a null context is refused."""
    import dataclasses
    from paper_1501_02565_amd import _lib
    from oracle import variational as va
    p = _lib.RefineParams()
    lib.epic_refine_defaults(ctypes.byref(p))
    for f in dataclasses.fields(va.Params):
        assert getattr(p, f.name) == pytest.approx(getattr(va.Params(), f.name), rel=1e-7), f.name
    assert (p.kappa, p.fixed_point, p.sor) == (5.0, 5, 30)
    for H, W, C in ((436, 1024, 3), (1, 1, 1), (97, 131, 4)):
        b = lib.epic_refine_bytes(H, W, C)
        assert 0 <= b - (104 + 4 * C) * H * W <= 27 * 256 + 256
    assert lib.epic_refine_bytes(0, 5, 3) == 0 and lib.epic_refine_bytes(5, 5, 5) == 0
    P = 0x1000
    assert lib.epic_refine(None, P, P, 10, 20, 3, P, P, None, None) == -1
