"""Second- and fourth-order splitting (Eq. split-op) on the GPU against the
oracle, for every schedule and precision; segment chaining and batching
with mixed splitting orders."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.metrics import report, within

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SUBSTEPS = {1: 1, 2: 1, 4: 3}          # transform round trips per step


def tol64(Nz, order):
    return 1e-12 + 1e-14 * Nz * SUBSTEPS[order]


def run(w, prec, order, schedule=None, zassenhaus=True):
    from paper_2201_08500_amd import Plan
    p = Plan.from_workload(w, precision=prec, schedule=schedule,
                           split_order=order, zassenhaus=zassenhaus)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = None if w.u is None else torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    a, b = p.propagate(E0, u)
    torch.cuda.synchronize()
    return a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128)


def oracle(w, prec, order, zassenhaus=True):
    E0 = w.E0_in if prec == "fp64" else w.E0_in.astype(np.complex64).astype(np.complex128)
    prob = O.Problem.from_workload(w, split_order=order, zassenhaus=zassenhaus)
    return O.march(prob, E0, w.u)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("schedule", ["stockham", "fourstep", "split"])
@pytest.mark.parametrize("prec", ["fp64", "fp32s", "fp32"])
@pytest.mark.parametrize("Nx", [1024, 2048])
def test_splitting_parity(order, schedule, prec, Nx):
    w = W.small(Nx=Nx, Nz=23, Nomega=3, seed=61 + Nx // 512)
    a, b = run(w, prec, order, schedule)
    ra, rb = oracle(w, prec, order)
    r = report(a, b, ra, rb)
    assert not within(r, tol64(w.Nz, order) if prec == "fp64" else 1e-5,
                      phase_tol=1e-10 if prec == "fp64" else 1e-4), r


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("Nx", [256, 512, 4096])
def test_splitting_parity_other_sizes(order, Nx):
    w = W.small(Nx=Nx, Nz=9, Nomega=2, seed=71)
    for prec in ("fp64", "fp32s"):
        a, b = run(w, prec, order)
        ra, rb = oracle(w, prec, order)
        r = report(a, b, ra, rb)
        assert not within(r, tol64(w.Nz, order) if prec == "fp64" else 1e-5), (prec, r)


@pytest.mark.parametrize("order", [2, 4])
def test_splitting_without_zassenhaus_and_with_slab(order):
    w = W.small(Nx=1024, Nz=17, Nomega=2, seed=73, x_front=-40e-6, thickness=120e-6)
    for schedule in ("fourstep", "split"):
        a, b = run(w, "fp64", order, schedule, zassenhaus=False)
        ra, rb = oracle(w, "fp64", order, zassenhaus=False)
        r = report(a, b, ra, rb)
        assert not within(r, tol64(w.Nz, order)), (schedule, r)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("schedule", ["fourstep", "split"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_splitting_segments_chain_bitwise(order, schedule, prec):
    """Segments [0,7) [7,19) [19,25) reproduce the monolithic march bitwise:
    each step is self-contained (its first B sub-step uses its own row)."""
    from paper_2201_08500_amd import Plan
    w = W.small(Nx=1024, Nz=25, Nomega=2, seed=75)
    p = Plan.from_workload(w, precision=prec, schedule=schedule, split_order=order)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = torch.from_numpy(w.u).cuda()
    table = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
    p.deformation_table(u, table)
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    p.march(E0, table, a, b)
    a1, b1 = torch.empty_like(E0), torch.empty_like(E0)
    p.march_segment(E0, None, table, 0, 7, a1, b1)
    p.march_segment(a1, b1, table, 7, 12, a1, b1)
    p.march_segment(a1, b1, table, 19, 6, a1, b1)
    torch.cuda.synchronize()
    assert torch.equal(a1, a) and torch.equal(b1, b)


def test_batch_with_mixed_orders_equals_alone():
    from paper_2201_08500_amd import Job, Plan, propagate_batch
    jobs, alone = [], []
    for i, (nx, order, prec) in enumerate([(1024, 1, "fp32s"), (1024, 2, "fp32s"),
                                           (2048, 4, "fp64"), (512, 2, "fp32"),
                                           (2048, 2, "fp32s"), (256, 4, "fp32s")]):
        w = W.small(Nx=nx, Nz=11 + i, Nomega=2 + i % 3, seed=80 + i)
        p = Plan.from_workload(w, precision=prec, split_order=order)
        E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
        u = torch.from_numpy(w.u).cuda()
        jobs.append(Job(p, E0, u))
        a, b = p.propagate(E0, u)
        alone.append((a, b))
    propagate_batch(jobs)
    torch.cuda.synchronize()
    for j, (a, b) in zip(jobs, alone):
        assert torch.equal(j.E0_out, a) and torch.equal(j.Eh_out, b)


@pytest.mark.parametrize("Nx", [256, 512])
@pytest.mark.parametrize("order", [1, 2, 4])
def test_split_schedule_small_sizes(Nx, order):
    """The split schedule at Nx 256 (one wavefront per envelope) and 512
    (two wavefronts per envelope, 256-point in-wavefront transform): parity
    for every precision and a general mask, and bitwise segment chaining."""
    from paper_2201_08500_amd import Plan
    w = W.small(Nx=Nx, Nz=19, Nomega=3, seed=120 + Nx // 256)
    for prec in ("fp64", "fp32s", "fp32"):
        a, b = run(w, prec, order, "split")
        ra, rb = oracle(w, prec, order)
        r = report(a, b, ra, rb)
        assert not within(r, tol64(w.Nz, order) if prec == "fp64" else 1e-5), (prec, r)
    x = (np.arange(Nx) - Nx // 2) * w.dx
    m = (x[None, :] >= (-10e-6 + 0.5 * np.arange(w.Nz) * w.dz)[:, None])
    p = Plan.from_workload(w, precision="fp64", schedule="split", split_order=order, mask=m)
    E0 = torch.from_numpy(w.E0_in).cuda()
    u = torch.from_numpy(w.u).cuda()
    a, b = p.propagate(E0, u)
    ra, rb = O.march(O.Problem.from_workload(w, split_order=order, mask=m), w.E0_in, w.u)
    r = report(a.cpu().numpy(), b.cpu().numpy(), ra, rb)
    assert not within(r, tol64(w.Nz, order)), r
    for prec in ("fp64", "fp32"):
        p = Plan.from_workload(w, precision=prec, schedule="split", split_order=order)
        E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
        table = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
        p.deformation_table(u, table)
        a, b = torch.empty_like(E0), torch.empty_like(E0)
        p.march(E0, table, a, b)
        a1, b1 = torch.empty_like(E0), torch.empty_like(E0)
        p.march_segment(E0, None, table, 0, 8, a1, b1)
        p.march_segment(a1, b1, table, 8, 11, a1, b1)
        torch.cuda.synchronize()
        assert torch.equal(a1, a) and torch.equal(b1, b), prec
