"""General crystal mask Pi(x, z) on the GPU: a slab-shaped mask reproduces
the slab march bitwise; shaped crystals (tilted entrance surface, wedge, a
Laue block with a hole) match the oracle for every schedule, precision and
splitting order; segments chain and batches mix masked and slab jobs."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.metrics import report, within

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def shaped_mask(w):
    """Tilted entrance surface x >= x_s(z) up to a wedge back face, plus a
    Laue block (all x) over a range of steps with a vacuum hole in it."""
    x = (np.arange(w.Nx) - w.Nx // 2) * w.dx
    z = np.arange(w.Nz) * w.dz
    xs = -30e-6 + 0.4 * z                      # tilted front surface
    xb = 60e-6 - 0.8 * z                       # wedge back face
    m = (x[None, :] >= xs[:, None]) & (x[None, :] < xb[:, None] + 80e-6)
    n1, n2 = w.Nz // 3, w.Nz // 3 + 5
    m[n1:n2] = True
    m[n1:n2, (x > 10e-6) & (x < 25e-6)] = False
    return m


def run(w, prec, mask=None, order=1, schedule=None, **kw):
    from paper_2201_08500_amd import Plan
    p = Plan.from_workload(w, precision=prec, schedule=schedule, split_order=order,
                           mask=mask, **kw)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = None if w.u is None else torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    a, b = p.propagate(E0, u)
    torch.cuda.synchronize()
    return a.cpu(), b.cpu()


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("schedule", ["stockham", "fourstep", "split"])
def test_slab_shaped_mask_is_bitwise_the_slab(order, schedule):
    w = W.small(Nx=1024, Nz=21, Nomega=2, seed=91, x_front=-15e-6, thickness=50e-6)
    x = (np.arange(w.Nx) - w.Nx // 2) * w.dx
    m = np.broadcast_to((x >= w.x_front) & (x < w.x_front + w.thickness), (w.Nz, w.Nx))
    for prec in ("fp64", "fp32s"):
        a1, b1 = run(w, prec, None, order, schedule)
        a2, b2 = run(w, prec, m, order, schedule)
        assert torch.equal(a1, a2) and torch.equal(b1, b2), prec


@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("schedule", ["stockham", "fourstep", "split"])
@pytest.mark.parametrize("prec", ["fp64", "fp32s", "fp32"])
def test_shaped_crystal_matches_oracle(order, schedule, prec):
    w = W.small(Nx=1024, Nz=30, Nomega=3, seed=93)
    m = shaped_mask(w)
    a, b = run(w, prec, m, order, schedule)
    E0 = w.E0_in if prec == "fp64" else w.E0_in.astype(np.complex64).astype(np.complex128)
    ra, rb = O.march(O.Problem.from_workload(w, mask=m, split_order=order), E0, w.u)
    r = report(a.numpy().astype(np.complex128), b.numpy().astype(np.complex128), ra, rb)
    sub = {1: 1, 2: 1, 4: 3}[order]
    assert not within(r, 1e-12 + 1e-14 * w.Nz * sub if prec == "fp64" else 1e-5), r


@pytest.mark.parametrize("Nx", [256, 512, 2048, 4096])
def test_shaped_crystal_other_sizes(Nx):
    w = W.small(Nx=Nx, Nz=14, Nomega=2, seed=95)
    m = shaped_mask(w)
    a, b = run(w, "fp64", m)
    ra, rb = O.march(O.Problem.from_workload(w, mask=m), w.E0_in, w.u)
    r = report(a.numpy(), b.numpy(), ra, rb)
    assert not within(r, 1e-12 + 1e-14 * w.Nz), r


@pytest.mark.parametrize("order", [1, 2])
def test_masked_segments_chain_bitwise(order):
    from paper_2201_08500_amd import Plan
    w = W.small(Nx=1024, Nz=24, Nomega=2, seed=97)
    m = shaped_mask(w)
    for schedule in ("fourstep", "split"):
        p = Plan.from_workload(w, precision="fp64", schedule=schedule, split_order=order,
                               mask=m)
        E0 = torch.from_numpy(w.E0_in).cuda()
        u = torch.from_numpy(w.u).cuda()
        table = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
        p.deformation_table(u, table)
        a, b = torch.empty_like(E0), torch.empty_like(E0)
        p.march(E0, table, a, b)
        a1, b1 = torch.empty_like(E0), torch.empty_like(E0)
        p.march_segment(E0, None, table, 0, 9, a1, b1)
        p.march_segment(a1, b1, table, 9, 15, a1, b1)
        torch.cuda.synchronize()
        assert torch.equal(a1, a) and torch.equal(b1, b), schedule


def test_batch_mixes_masked_and_slab_jobs():
    from paper_2201_08500_amd import Job, Plan, propagate_batch
    jobs, alone = [], []
    for i, (nx, masked) in enumerate([(1024, True), (1024, False), (2048, True),
                                      (512, False), (2048, False), (512, True)]):
        w = W.small(Nx=nx, Nz=10 + i, Nomega=2, seed=100 + i)
        p = Plan.from_workload(w, precision="fp32s", mask=shaped_mask(w) if masked else None)
        E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
        u = torch.from_numpy(w.u).cuda()
        jobs.append(Job(p, E0, u))
        alone.append(p.propagate(E0, u))
    propagate_batch(jobs)
    torch.cuda.synchronize()
    for j, (a, b) in zip(jobs, alone):
        assert torch.equal(j.E0_out, a) and torch.equal(j.Eh_out, b)
