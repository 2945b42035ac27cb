"""Host-side checks of the C-ABI library (no GPU calls): it loads, exports
every function include/lbm.h declares, and its struct layouts match the
header's field order and sizes."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="lbm.h", prefix="lbm_"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lbm_create", "lbm_step", "lbm_particles_sync", "lbm_fields", "lbm_destroy",
              "lbm_last_error", "lbm_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2505_10171_amd import lbm
    L = lbm.load_library()
    for n in _declared():
        assert hasattr(L, n), n
    assert sorted(lbm.EXPORTS) == _declared()


def test_library_exports_every_surrogate_symbol():
    from paper_2505_10171_amd import surrogate
    L = surrogate.library()
    names = _declared("srg.h", "srg_")
    assert "srg_train" in names and "srg_predict" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(surrogate.SRG_EXPORTS) == names


def test_surrogate_parameter_count_and_workspace():
    from oracle.surrogate_oracle import SIZES
    from paper_2505_10171_amd import surrogate
    n = sum(a * b + b for a, b in zip(SIZES[:-1], SIZES[1:]))
    assert n == surrogate.SRG_PARAMS == 212275
    hdr = open(os.path.join(ROOT, "include", "srg.h")).read()
    assert "#define SRG_PARAMS 212275" in hdr
    L = surrogate.library()
    assert L.srg_workspace_bytes(100, 10) == 0  # batch not a multiple of 64
    assert L.srg_workspace_bytes(1024, 4096) > 4 * 4 * n


def _c_layout(struct, fields, tmp_path):
    """sizeof/offsetof of a header struct, printed by a C program built with gcc."""
    import subprocess
    src = tmp_path / "lay.c"
    body = "".join(f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\n'
                   f'int main(void){{printf("%zu\\n", sizeof({struct}));{body}return 0;}}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("name", ["LbmConfig", "LbmParticle"])
def test_struct_layout_matches_header(name, tmp_path):
    from paper_2505_10171_amd import lbm
    cls = getattr(lbm, name)
    cname = {"LbmConfig": "lbm_config", "LbmParticle": "lbm_particle"}[name]
    fields = [f for f, _ in cls._fields_]
    got = _c_layout(cname, fields, tmp_path)
    assert got[0] == C.sizeof(cls)
    assert got[1:] == [getattr(cls, f).offset for f in fields]


def test_workspace_sizing_and_validation():
    """lbm_workspace_bytes is pure host arithmetic: it validates the
    configuration and sizes the workspace (two population buffers dominate)."""
    from paper_2505_10171_amd import lbm, workloads as W
    L = lbm.load_library()
    cfg = W.config(64, 32, 16)
    c = (lbm.LbmConfig * 1)(lbm.make_config(cfg, 0))
    nb = L.lbm_workspace_bytes(c, 1, None, 0)
    N = 64 * 32 * 16
    # per node besides the two population buffers (19 values per node, padded
    # to 64 nodes): moments (rho, phi) of two states 16 B, interface normal
    # 16 B, curvature term + solid-link bits 8 B, mask 2 B, claim 4 B
    assert nb >= 2 * 19 * 4 * N + 46 * N
    assert nb < 2 * 19 * 4 * N + 48 * N + 64 * 19 * 4 * 2 + 4096
    bad = dict(cfg, tau_a=0.5)
    c = (lbm.LbmConfig * 1)(lbm.make_config(bad, 0))
    assert L.lbm_workspace_bytes(c, 1, None, 0) == 0
    bad = dict(cfg, theta_wall_deg=180.0)
    c = (lbm.LbmConfig * 1)(lbm.make_config(bad, 0))
    assert L.lbm_workspace_bytes(c, 1, None, 0) == 0
    # open x ends and the tube wall: kinds and boundary densities are checked
    for bad in (dict(cfg, has_wall=4), dict(cfg, has_wall=2, tube_R=0.0),
                dict(cfg, open_x=1, rho_in=0.0), dict(cfg, open_x=1, rho_out=-1.0),
                dict(cfg, open_x=2), dict(cfg, has_wall=3, boxes=[(0, 0, 1, 64, 3, 3)]),
                dict(cfg, has_wall=3, boxes=[(5, 0, 1, 4, 3, 3)]),
                dict(cfg, has_wall=3, boxes=[(0, 0, 1, 3, 3, 3)] * 9),
                dict(cfg, has_wall=3, open_x=1, boxes=[(0, 0, 1, 3, 3, 3)])):
        c = (lbm.LbmConfig * 1)(lbm.make_config(bad, 0))
        assert L.lbm_workspace_bytes(c, 1, None, 0) == 0, bad
    ok = dict(cfg, has_wall=2, tube_R=7.5, open_x=1, rho_in=0.051, rho_out=0.049)
    c = (lbm.LbmConfig * 1)(lbm.make_config(ok, 0))
    assert L.lbm_workspace_bytes(c, 1, None, 0) == nb
    ok = dict(cfg, has_wall=3, boxes=[(0, 0, 1, 63, 31, 3), (10, 10, 4, 12, 12, 9)])
    c = (lbm.LbmConfig * 1)(lbm.make_config(ok, 0))
    assert L.lbm_workspace_bytes(c, 1, None, 0) == nb
    # FP16 storage halves the population bytes
    c16 = (lbm.LbmConfig * 1)(lbm.make_config(dict(cfg, storage="fp16"), 0))
    assert L.lbm_workspace_bytes(c16, 1, None, 0) < 0.5 * (nb - 46 * N) + 48 * N + 4096


def test_error_paths_without_gpu():
    from paper_2505_10171_amd import lbm
    L = lbm.load_library()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_last_error(None) is None
    out = C.c_void_p()
    assert L.lbm_create(None, 1, None, None, 0, None, 0, None, C.byref(out)) == lbm.LBM_EINVAL
    L.lbm_destroy(out)
