"""lbm_moments_f64_noalloc, the readout for callers that cannot allocate,
against lbm_moments_f64 through the C ABI: the same bits on two calls in a
row (the second on a smaller instance), after a fused last launch (whose
earlier steps the readout replays) and after a single step, and the size
limit refused with nothing written."""
import numpy as np
import pytest

import workloads as W
import paper_2010_01847_amd as P
from paper_2010_01847_amd import LBMError, LBM_EINVAL, Lattice, instance_from_case

pytestmark = pytest.mark.gpu


def _case(nx, ny, seed, **kw):
    case = W.Case(f"noalloc_{nx}x{ny}", nx, ny, 0.6, 7.0, **kw)
    T0 = W.random_field(nx, ny, 0.01, case.t0, seed) + (np.tile(case.t_ref(), (ny, 1)) - case.t0)
    qx, qy = W.random_flux(nx, ny, 1e-3, seed + 1)
    return case, T0, qx, qy


@pytest.mark.parametrize("storage", ["f32", "f16_split"])
def test_noalloc_readout_equals_moments_f64(storage):
    big, Tb, qxb, qyb = _case(1000, 1048, 3)                 # 1,048,000 nodes: just under 2^20
    small, Ts, qxs, qys = _case(77, 53, 5, bc_y="diffuse")
    lat = Lattice([instance_from_case(big), instance_from_case(small)], storage=storage, check_interval=10)
    lat.set_step_fusion(P.lbm_max_step_fusion(P.STORAGE[storage]))
    lat.init(0, Tb, qxb, qyb)
    lat.init(1, Ts, qxs, qys)
    for n in (23, 1, 16):                     # ends: a fused launch, a single step, a fused check launch
        lat.step(n)
        for k in (0, 1):                      # two calls in a row, the second smaller
            want = lat.moments(k)
            got = lat.moments_noalloc(k)
            for a, b in zip(got, want):
                assert a.shape == b.shape
                assert np.array_equal(a, b), (storage, lat.steps, k)
        # only some fields asked for: the others stay untouched
        it = lat.instances[1]
        qx_only = np.empty((it.ny, it.nx))
        P.lbm_moments_f64_noalloc(lat.h, 1, 0, qx_only.ctypes.data, 0)
        assert np.array_equal(qx_only, lat.moments(1)[1])
    lat.close()


def test_noalloc_readout_refuses_large_instances():
    case = W.Case("noalloc_large", 1025, 1024, 0.6, 7.0)    # 2^20 + 1024 nodes
    lat = Lattice([instance_from_case(case)], check_interval=-1)
    lat.init(0)
    lat.step(2)
    out = np.full((case.ny, case.nx), 7.0)
    with pytest.raises(LBMError) as e:
        P.lbm_moments_f64_noalloc(lat.h, 0, out.ctypes.data, 0, 0)
    assert e.value.code == LBM_EINVAL
    assert np.all(out == 7.0)
    lat.close()
