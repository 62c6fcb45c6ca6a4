"""bpm_propagate_noalloc (static device workspace, no allocation by the call)
against bpm_propagate through the C ABI: the same kernels on the same
inputs, so the outputs must be bitwise equal -- on two calls in a row, the
second with a smaller problem (the array keeps the first call's contents),
for a plan that has and one that has not uploaded its constants, with a
general crystal mask, in every precision; and a problem larger than the
static array is refused."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _inputs(p, w):
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = None if w.u is None else torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    return E0, u


def _both(w, prec, **kw):
    """(bpm_propagate result, bpm_propagate_noalloc result) of one problem;
    the no-alloc call runs on a fresh plan first (constants staged in the
    static array), then bpm_propagate on another plan."""
    from paper_2201_08500_amd import Plan
    pn = Plan.from_workload(w, precision=prec, **kw)
    E0, u = _inputs(pn, w)
    a = torch.full_like(E0, 7.0)
    b = torch.full_like(E0, -7.0)
    pn.propagate_noalloc(E0, u, a, b)
    pr = Plan.from_workload(w, precision=prec, **kw)
    ra, rb = pr.propagate(E0, u)
    torch.cuda.synchronize()
    return (ra, rb), (a, b), pn


@pytest.mark.parametrize("prec", ["fp64", "fp32s", "fp32"])
def test_noalloc_equals_propagate_two_calls_second_smaller(prec):
    big = W.small(Nx=2048, Nz=60, Nomega=6, seed=401)
    small = W.small(Nx=512, Nz=25, Nomega=2, seed=402)
    (ra, rb), (a, b), _ = _both(big, prec)
    assert torch.equal(a, ra) and torch.equal(b, rb)
    (ra, rb), (a, b), _ = _both(small, prec)
    assert torch.equal(a, ra) and torch.equal(b, rb)


def test_noalloc_after_the_plan_uploaded_its_constants():
    """A plan that has run bpm_propagate keeps its uploaded constants; the
    no-alloc call then uses them and stages only the table."""
    from paper_2201_08500_amd import Plan
    w = W.small(Nx=1024, Nz=40, Nomega=3, seed=403)
    p = Plan.from_workload(w, precision="fp32s")
    E0, u = _inputs(p, w)
    ra, rb = p.propagate(E0, u)
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    for _ in range(2):
        a.fill_(3.0)
        b.fill_(3.0)
        p.propagate_noalloc(E0, u, a, b)
        torch.cuda.synchronize()
        assert torch.equal(a, ra) and torch.equal(b, rb)


def test_noalloc_undeformed_and_masked():
    w = W.small(Nx=1024, Nz=30, Nomega=2, seed=404, deformed=False)
    (ra, rb), (a, b), _ = _both(w, "fp64")
    assert torch.equal(a, ra) and torch.equal(b, rb)
    w = W.small(Nx=1024, Nz=30, Nomega=2, seed=405)
    x = (np.arange(w.Nx) - w.Nx // 2) * w.dx
    m = x[None, :] >= (-30e-6 + 0.3 * np.arange(w.Nz) * w.dz)[:, None]
    (ra, rb), (a, b), _ = _both(w, "fp32s", mask=m, split_order=2)
    assert torch.equal(a, ra) and torch.equal(b, rb)


def test_noalloc_refuses_problems_beyond_the_static_array():
    from paper_2201_08500_amd import BpmError, Plan
    from paper_2201_08500_amd._native import NOALLOC_MAX_BYTES
    # 4096 x 4096 cells of complex128 table = 256 MiB > 128 MiB
    w = W.small(Nx=4096, Nz=4096, Nomega=1, seed=406, deformed=False)
    p = Plan.from_workload(w, precision="fp64")
    assert p.Nx * p.Nz * 16 > NOALLOC_MAX_BYTES
    E0 = torch.from_numpy(w.E0_in).cuda()
    u = torch.zeros(w.Nz, w.Nx, dtype=torch.float64, device="cuda")
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    with pytest.raises(BpmError, match="static workspace"):
        p.propagate_noalloc(E0, u, a, b)
