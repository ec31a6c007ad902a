"""Host-side checks of the gfx950 library (no GPU needed, no kernel calls).

The C-ABI library must load and export every function include/lbmep.h
declares; the Python binding must declare the same set; host-only argument
checks (configuration validation, footprint) behave as documented.
"""
import ctypes
import os
import re

import pytest

from paper_1708_08741_amd import lbmep as lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lbmep.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbmep_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = lb.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/lbmep.h but not exported"
    assert sorted(lb.exported_symbols()) == names


def test_config_struct_layout():
    # int32 nx,ny,nz, periodic[3]; double nu, magic; int32 precision,
    # move_particles, device, reserved; void* stream
    assert ctypes.sizeof(lb.Config) == 64
    assert lb.Config.nu.offset == 24 and lb.Config.stream.offset == 56


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and offsets a C
    compiler gives the header's structures."""
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "lbmep.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu\\n", sizeof(lbmep_config), sizeof(lbmep_server_config),'
        " sizeof(lbmep_request), sizeof(lbmep_server_stats));\n"
        '  printf("%zu %zu %zu %zu %zu\\n", offsetof(lbmep_request, flags),'
        " offsetof(lbmep_request, X), offsetof(lbmep_request, rho_e),"
        " offsetof(lbmep_request, E), offsetof(lbmep_server_stats, cell_updates_done));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split()
    sizes = [int(v) for v in out[:4]]
    offs = [int(v) for v in out[4:]]
    assert sizes == [ctypes.sizeof(lb.Config), ctypes.sizeof(lb.ServerConfig),
                     ctypes.sizeof(lb.Request), ctypes.sizeof(lb.ServerStats)]
    assert offs == [lb.Request.flags.offset, lb.Request.X.offset, lb.Request.rho_e.offset,
                    lb.Request.E.offset, lb.ServerStats.cell_updates_done.offset]


def test_server_request_footprint_host_only():
    """Admission footprint of a request: the lattice's footprint plus the
    arena alignment, descriptor and set-up staging; checked on the host."""
    import numpy as np
    shape = (64, 96, 128)
    N = 64 * 96 * 128
    kw = dict(X=np.array([[10.0, 10.0, 10.0]]), R=[4.0], U=np.zeros((1, 3)), steps=100,
              rho_e=np.zeros(N, dtype=np.float32), E=(1e-3, 0, 0), precision=lb.FP32DEV)
    fp = lb.Server.request_footprint(shape, **kw)
    base = lb.footprint(shape, lb.FP32DEV, 1, True)
    assert base < fp < base + 8 * N + 64 * 4096
    fp_keep = lb.Server.request_footprint(shape, keep_fields=True, **kw)
    assert fp_keep - fp >= 32 * N
    with pytest.raises(lb.LbmepError) as e:
        lb.Server.request_footprint((0, 4, 4), steps=1)
    assert e.value.code == lb.EINVAL


def test_library_is_gfx950_only():
    """The shared object carries gfx950 device code and no other target."""
    data = open(lb.LIB_PATH, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx90a", b"gfx942", b"gfx1100", b"sm_"):
        assert other + b"\x00" not in data or other == b"sm_"


@pytest.mark.parametrize("shape,prec,np_,charge", [
    ((512, 512, 512), lb.FP32DEV, 4096, True),
    ((512, 512, 512), lb.FP16DEV, 4096, True),
    ((512, 512, 512), lb.FP64, 0, False),
    ((64, 96, 128), lb.FP32DEV, 200, True),
])
def test_footprint(shape, prec, np_, charge):
    """Footprint = two population grids + flags/masks (+ maps, force, the
    particles' link lists, which grow with the largest radius)."""
    b = lb.footprint(shape, prec, np_, charge, r_max=4.0)
    N = shape[0] * shape[1] * shape[2]
    es = {lb.FP64: 8, lb.FP32DEV: 4, lb.FP16DEV: 2}[prec]
    pops = 2 * 19 * N * es
    links = np_ * (8 * 11 ** 3 + 4)  # (2 ceil(R) + 3)^3 entries of 8 bytes per particle
    assert pops + links < b < pops + links + 18 * N + 8 * N + 10_000_000
    if np_:
        assert lb.footprint(shape, prec, np_, charge, r_max=8.0) - b == np_ * 8 * (19 ** 3 - 11 ** 3)
    if shape == (512, 512, 512) and prec == lb.FP32DEV:
        assert 20.4e9 < b < 24e9  # fits one MI355X (288 GB) many times over
    if np_:
        # moving particles: the next level's link lists of the overlapped step
        bm = lb.footprint(shape, prec, np_, charge, r_max=4.0, move_particles=True)
        assert bm - b == links


@pytest.mark.parametrize("kw", [
    dict(shape=(0, 4, 4)), dict(shape=(4, -1, 4)), dict(shape=(4, 4, 4), nu=0.0),
    dict(shape=(4, 4, 4), nu=float("nan")), dict(shape=(4, 4, 4), magic=0.0),
    dict(shape=(4, 4, 4), precision=7), dict(shape=(4, 4, 70000)),
])
def test_config_validation(kw):
    shape = kw.pop("shape")
    prec = kw.pop("precision", lb.FP64)
    with pytest.raises(lb.LbmepError) as e:
        lb.footprint(shape, prec, 0, False, **kw)
    assert e.value.code == lb.EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(lb, "_lib", None)
    monkeypatch.setattr(lb, "LIB_PATH", str(tmp_path / "liblbmep.so"))
    with pytest.raises(ImportError):
        lb.lib()
