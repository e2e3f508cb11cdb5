"""dgw_step_ader_noalloc through the C ABI against dgw_step_ader: the same
kernels with the work registers in the library's static device scratch
instead of a caller's work buffer.  Two calls in a row, the second on a
smaller input; a size beyond the scratch is rejected before any launch."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def test_noalloc_ader_equals_step_ader(gpu_lib):
    B = gpu_lib
    say("noalloc: 3D 4^3 k=4, batch of 2 with sources, 3 steps")
    big = B.Mesh(3, 4, W.box_nodes(3, 4, 4, 0.05), W.box_neighbors(3, 4),
                 W.FourierMaterial(5, dim=3, rho_amp=0.3), max_batch=2)
    U = W.random_state(71, (2,) + big.shape)
    src = B.Sources(big, W.random_points(72, 2, 3), frequency=6.0)
    dt = 0.2 * big.info.dt_unit
    a, b = to_dev(U), to_dev(U)
    big.step_ader(a, 0.1, dt, 3, sources=src, B=2)
    big.step_ader_noalloc(b, 0.1, dt, 3, sources=src, B=2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    say("noalloc: 2D 5^2 k=3, one member, 2 steps (smaller input, same scratch)")
    small = B.Mesh(2, 3, W.box_nodes(2, 5, 3, 0.05), W.box_neighbors(2, 5), W.FourierMaterial(6, dim=2, rho_amp=0.3))
    V = W.random_state(73, (1,) + small.shape)
    a, b = to_dev(V), to_dev(V)
    dt = 0.3 * small.info.dt_unit
    small.step_ader(a, 0.0, dt, 2)
    small.step_ader_noalloc(b, 0.0, dt, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # the HDG-ADER variant goes through the same scratch
    a, b = to_dev(V), to_dev(V)
    small.step_ader(a, 0.0, dt, 1, flags=B.ADER_HDG)
    small.step_ader_noalloc(b, 0.0, dt, 1, flags=B.ADER_HDG)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_noalloc_rejects_what_it_cannot_hold(gpu_lib):
    B = gpu_lib
    say("noalloc: size and level checks")
    m = B.Mesh(3, 5, W.box_nodes(3, 8, 5, 0.05), W.box_neighbors(3, 8), W.ConstantMaterial(), max_batch=10)
    u = torch.zeros((10,) + m.shape, dtype=torch.float64, device="cuda")
    assert 2 * 10 * m.info.state_bytes > 64 << 20
    with pytest.raises(B.DgwError) as e:
        m.step_ader_noalloc(u, 0.0, 1e-3, 1, B=10)
    assert e.value.status == B.EINVAL
    # the every-third reduction needs its reduced levels: built by one dgw_step_ader
    v = torch.zeros((1,) + m.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(B.DgwError) as e:
        m.step_ader_noalloc(v, 0.0, 1e-3, 1, flags=B.ADER_REDUCE_EVERY_THIRD)
    assert e.value.status == B.EUNSUPPORTED
    w = torch.ones((1,) + m.shape, dtype=torch.float64, device="cuda")
    x = w.clone()
    m.step_ader(w, 0.0, 1e-3, 1, flags=B.ADER_REDUCE_EVERY_THIRD)
    m.step_ader_noalloc(x, 0.0, 1e-3, 1, flags=B.ADER_REDUCE_EVERY_THIRD)
    torch.cuda.synchronize()
    assert torch.equal(w, x)
