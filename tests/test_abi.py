"""The C ABI library loads on a machine without a GPU and exports every entry
point the header declares; host-side validation answers without a device."""
import ctypes
import math
import os
import re

import pytest

import paper_2010_01847_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phonon_lbm.h")
HEADER3 = os.path.join(ROOT, "include", "phonon_d3q14.h")


def _declared(path=HEADER, prefix="lbm_"):
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = _declared()
    assert "lbm_create" in names and "lbm_step" in names and "lbm_residual" in names
    L = P.library()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    bound = {s[0] for s in P.lbm.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def test_d3q14_header_symbols_exported():
    names = _declared(HEADER3, "lbm3d_")
    assert "lbm3d_create" in names and "lbm3d_step" in names and "lbm3d_sample" in names
    L = P.d3q14.library()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == {s[0] for s in P.d3q14.SIGNATURES3}
    # every header under include/ is covered by one of the two binding tables
    inc = os.path.join(ROOT, "include")
    assert sorted(os.listdir(inc)) == ["phonon_d3q14.h", "phonon_lbm.h"]


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes structs equal those a C compiler
    gives the header's structs."""
    import subprocess
    structs = {"lbm_instance": P.lbm_instance, "lbm_config": P.lbm_config,
               "lbm_check_info": P.lbm_check_info, "lbm_launch_shape": P.lbm_launch_shape,
               "lbm3d_config": P.d3q14.lbm3d_config, "lbm3d_launch_shape": P.d3q14.lbm3d_launch_shape}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "phonon_lbm.h"', '#include "phonon_d3q14.h"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


def _cfg(insts, storage=P.LBM_F32, check=0, flags=P.LBM_FLAG_EXTERNAL_MEMORY):
    arr = (P.lbm_instance * len(insts))(*insts)
    cfg = P.lbm_config()
    cfg.n_instances = len(insts)
    cfg.storage = storage
    cfg.check_interval = check
    cfg.flags = flags
    cfg.inst = ctypes.cast(arr, ctypes.POINTER(P.lbm_instance))
    cfg._keep = arr
    return cfg


def test_required_bytes_and_layout():
    it = P.make_instance(100, 30, 0.6, 0.8)
    b32 = P.lbm_required_bytes(_cfg([it], check=-1))
    b16 = P.lbm_required_bytes(_cfg([it], storage=P.LBM_F16, check=-1))
    # two buffers of 8 planes, rows padded to 256 bytes
    assert b32 >= 2 * 8 * 30 * 128 * 4
    assert b16 >= 2 * 8 * 30 * 128 * 2
    assert b32 > b16
    # check-step snapshot adds 3 doubles per node
    assert P.lbm_required_bytes(_cfg([it], check=10)) - b32 >= 3 * 8 * 100 * 30
    # split storage: per 64-node chunk eight 16-bit runs plus one FP32 energy
    # run (1280 bytes), chunked layout only
    bs = P.lbm_required_bytes(_cfg([it], storage=P.LBM_F16_SPLIT, check=-1))
    assert bs >= 2 * 30 * 2 * 1280
    assert bs - P.lbm_required_bytes(_cfg([it], storage=P.LBM_BF16_SPLIT, check=-1)) == 0
    cfg = _cfg([it], storage=P.LBM_BF16_SPLIT, check=-1)
    cfg.layout = P.LBM_LAYOUT_PLANES
    with pytest.raises(P.LBMError) as e:
        P.lbm_required_bytes(cfg)
    assert e.value.code == P.LBM_EUNSUPPORTED


@pytest.mark.parametrize("kw,code", [
    (dict(nx=1, ny=8, tau_n=0.6, tau_r=0.8), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.0, tau_r=0.8), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=-1.0), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=math.inf, tau_r=1.0), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x="diffuse", bc_y="isothermal"), P.LBM_EUNSUPPORTED),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x="isothermal", bc_y="diffuse", wall_bc=(0, "heatflux", 0, 0)),
     P.LBM_EUNSUPPORTED),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, wall_bc=(0, 0, "isothermal", 0)), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_y="diffuse", wall_bc=(0, 0, "gradient", 0)), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x="gradient", bc_y="diffuse", wall_bc=(0, 0, 0, "isothermal")),
     P.LBM_EUNSUPPORTED),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x="gradient", bc_y="isothermal"), P.LBM_EUNSUPPORTED),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_y=P.LBM_BC_GRADIENT), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, scale=3.0), P.LBM_EINVAL),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x="heatflux", bc_y="diffuse"), P.LBM_EUNSUPPORTED),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x="heatflux", bc_y="isothermal"), P.LBM_EUNSUPPORTED),
    (dict(nx=8, ny=8, tau_n=0.6, tau_r=0.8, bc_x=5), P.LBM_EINVAL),
])
def test_config_validation(kw, code):
    with pytest.raises(P.LBMError) as e:
        P.lbm_required_bytes(_cfg([P.make_instance(**kw)]))
    assert e.value.code == code


def test_bad_config_fields():
    it = P.make_instance(8, 8, 0.6, 0.8)
    for field, val in (("storage", 7), ("check_interval", 1), ("flags", 0x100)):
        cfg = _cfg([it])
        setattr(cfg, field, val)
        with pytest.raises(P.LBMError) as e:
            P.lbm_required_bytes(cfg)
        assert e.value.code == P.LBM_EINVAL
    cfg = _cfg([it])
    cfg.n_instances = 0
    with pytest.raises(P.LBMError):
        P.lbm_required_bytes(cfg)


def test_heatflux_pairs_accepted():
    for bx, by in (("heatflux", "periodic"), ("periodic", "heatflux"), ("gradient", "heatflux")):
        assert P.lbm_required_bytes(_cfg([P.make_instance(16, 8, 0.6, 0.8, bc_x=bx, bc_y=by)])) > 0


def test_per_wall_kinds_and_corners_accepted():
    """Mixed kinds on one axis, and walls on both axes when both x walls are
    isothermal (they own the corners; the Sec. 3.1.2 square)."""
    for kw in (dict(bc_x="isothermal", bc_y="isothermal", wall_bc=(0, 0, 0, "heatflux")),
               dict(bc_x="isothermal", bc_y="diffuse"),
               dict(bc_y="diffuse", wall_bc=(0, 0, "isothermal", "heatflux")),
               dict(bc_x="gradient", bc_y="diffuse", wall_bc=(0, 0, "heatflux", 0))):
        assert P.lbm_required_bytes(_cfg([P.make_instance(16, 8, 0.6, 0.8, **kw)])) > 0


def test_tau_r_infinite_and_small_accepted():
    for tr in (math.inf, 0.2, 1e6):
        assert P.lbm_required_bytes(_cfg([P.make_instance(16, 8, 0.6, tr)])) > 0


def test_max_step_fusion_per_storage_kind():
    """The most time steps per fused launch, per storage kind (no device)."""
    got = [P.lbm_max_step_fusion(k) for k in (P.LBM_F32, P.LBM_F16, P.LBM_BF16, P.LBM_F16_SPLIT,
                                               P.LBM_BF16_SPLIT)]
    assert got == [7, 6, 6, 6, 6]
    assert P.lbm_max_step_fusion(5) == -1 and P.lbm_max_step_fusion(-1) == -1


def test_round_every_step_flag_accepted():
    """LBM_FLAG_ROUND_EVERY_STEP is a known flag for every storage kind."""
    for st in (P.LBM_F32, P.LBM_F16, P.LBM_BF16_SPLIT):
        cfg = _cfg([P.make_instance(70, 33, 0.6, 5.0)], storage=st,
                   flags=P.LBM_FLAG_EXTERNAL_MEMORY | P.LBM_FLAG_ROUND_EVERY_STEP)
        assert P.lbm_required_bytes(cfg) > 0


def test_readout_region_sized_for_moment_planes():
    """16-bit storage rounding only the stored step rebuilds readouts as FP64
    moment planes (24 bytes per node) instead of a population buffer (16 or
    20 bytes per node on rows of whole 64-node chunks): its handles need more
    memory than with LBM_FLAG_ROUND_EVERY_STEP, by about 24 - 20 bytes per node
    or more; FP32 handles need the same either way."""
    insts = [P.make_instance(1024, 700, 0.6, 5.0), P.make_instance(384, 129, 0.7, 50.0)]
    nodes = 1024 * 700 + 384 * 129
    every = P.LBM_FLAG_EXTERNAL_MEMORY | P.LBM_FLAG_ROUND_EVERY_STEP
    for st in (P.LBM_F16, P.LBM_BF16, P.LBM_F16_SPLIT, P.LBM_BF16_SPLIT):
        dflt = P.lbm_required_bytes(_cfg(insts, storage=st))
        flag = P.lbm_required_bytes(_cfg(insts, storage=st, flags=every))
        assert dflt - flag >= 3.9 * nodes, st
    assert P.lbm_required_bytes(_cfg(insts)) == P.lbm_required_bytes(_cfg(insts, flags=every))


def test_null_handle_calls_are_rejected():
    assert P.library().lbm_step(None, 1) == P.LBM_EINVAL
    assert P.library().lbm_steps_done(None) == -1
    assert P.library().lbm_set_streams(None, 2) == P.LBM_EINVAL
    assert P.library().lbm_get_streams(None) == -1
    P.library().lbm_destroy(None)   # ignored


# ---------------------------------------------------------------- D3Q14

def _cfg3(**kw):
    c = P.d3q14.lbm3d_config()
    c.nx, c.ny, c.nz = kw.get("nx", 16), kw.get("ny", 8), kw.get("nz", 4)
    c.storage = kw.get("storage", P.LBM_F32)
    c.flags = kw.get("flags", P.LBM_FLAG_EXTERNAL_MEMORY)
    c.layout = kw.get("layout", P.LBM_LAYOUT_AUTO)
    c.tau_n, c.tau_r = kw.get("tau_n", 0.6), kw.get("tau_r", 0.8)
    c.cv, c.t0, c.scale = kw.get("cv", 1.0), kw.get("t0", 1.0), kw.get("scale", 0.0)
    return c


@pytest.mark.parametrize("layout", [P.LBM_LAYOUT_PLANES, P.LBM_LAYOUT_CHUNKED, P.LBM_LAYOUT_AUTO])
def test_d3q14_required_bytes(layout):
    """Two buffers of 14 populations per node, rows padded to 64 nodes."""
    b32 = P.d3q14.lbm3d_required_bytes(_cfg3(nx=100, ny=30, nz=7, layout=layout))
    b16 = P.d3q14.lbm3d_required_bytes(_cfg3(nx=100, ny=30, nz=7, storage=P.LBM_BF16, layout=layout))
    assert b32 >= 2 * 14 * 128 * 30 * 7 * 4
    assert b16 >= 2 * 14 * 128 * 30 * 7 * 2 and b16 < b32
    assert P.d3q14.lbm3d_required_bytes(_cfg3(nx=1, ny=1, nz=1)) > 0


@pytest.mark.parametrize("kw", [
    dict(nx=0), dict(ny=0), dict(nz=-1), dict(tau_n=0.0), dict(tau_n=math.inf), dict(tau_r=0.0),
    dict(tau_r=-2.0), dict(storage=P.LBM_F16_SPLIT), dict(storage=9), dict(flags=0x100),
    dict(scale=3.0), dict(scale=-1.0), dict(cv=-1.0), dict(t0=math.nan),
    dict(nx=4096, ny=4096, nz=256),           # 2^32 nodes
    dict(layout=3),
])
def test_d3q14_config_validation(kw):
    with pytest.raises(P.LBMError) as e:
        P.d3q14.lbm3d_required_bytes(_cfg3(**kw))
    assert e.value.code == P.LBM_EINVAL


@pytest.mark.parametrize("n,storage,fuse", [(128, P.LBM_F32, 1), (192, P.LBM_F32, 2), (512, P.LBM_F32, 2),
                                             (128, P.LBM_F16, 1), (512, P.LBM_F16, 2), (512, P.LBM_BF16, 2)])
def test_d3q14_default_step_fusion(n, storage, fuse):
    """Two steps per launch by default, for every storage kind, for boxes
    holding at least 256 two-step blocks (60 x 12 x 32 nodes): 128^3 holds
    132, 192^3 384."""
    D = P.d3q14
    h = D.lbm3d_create(_cfg3(nx=n, ny=n, nz=n, storage=storage))
    try:
        assert D.lbm3d_get_step_fusion(h) == fuse
    finally:
        D.lbm3d_destroy(h)


def test_d3q14_handle_state_without_gpu():
    """Create and bind take no device action with external memory; stepping
    before init and bad launch shapes are rejected on the host."""
    D = P.d3q14
    h = D.lbm3d_create(_cfg3(tau_r=math.inf))
    try:
        with pytest.raises(P.LBMError) as e:
            D.lbm3d_step(h, 1)
        assert e.value.code == P.LBM_ESTATE
        with pytest.raises(P.LBMError) as e:
            D.lbm3d_bind(h, 0x1000 + 3, 1 << 40)
        assert e.value.code == P.LBM_EINVAL
        for bad in ((3, 1, 0, 1, 8), (4, 2, 0, 1, 8), (1, 0, 5, 1, 8), (1, 0, 0, 3, 8), (2, 0, 0, 8, 8),
                    (1, 0, 0, 0, 8), (1, 0, 0, 1, 0)):
            with pytest.raises(P.LBMError):
                D.lbm3d_set_launch_shape(h, D.lbm3d_launch_shape(*bad))
        D.lbm3d_set_launch_shape(h, D.lbm3d_launch_shape(2, 0, 1, 4, 16))
        s = D.lbm3d_get_launch_shape(h)
        assert (s.rows_per_tile, s.xcd_remap, s.nontemporal, s.tile_waves, s.zchunk) == (2, 0, 1, 4, 16)
        for bad in (0, 3):
            with pytest.raises(P.LBMError):
                D.lbm3d_set_step_fusion(h, bad)
        assert D.lbm3d_get_step_fusion(h) == 1        # 16 x 8 x 4: too few two-step blocks
        D.lbm3d_set_step_fusion(h, 2)
        assert D.lbm3d_get_step_fusion(h) == 2
        assert D.lbm3d_steps_done(h) == 0
        with pytest.raises(P.LBMError) as e:
            D.lbm3d_autotune(h, 2)           # no memory bound yet
        assert e.value.code == P.LBM_ESTATE
    finally:
        D.lbm3d_destroy(h)
    assert P.d3q14.library().lbm3d_step(None, 1) == P.LBM_EINVAL
    assert P.d3q14.library().lbm3d_steps_done(None) == -1
    assert P.d3q14.library().lbm3d_get_step_fusion(None) == -1
    P.d3q14.library().lbm3d_destroy(None)
