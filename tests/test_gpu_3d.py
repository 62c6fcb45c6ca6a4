"""GPU parity of the march on a 3D grid (bpm_plan_create_3d) against the FP64
3D oracle: power-of-two x lengths (direct transform) and others (cyclic
convolution on a padded length), odd and even Ny up to the maximum, every
precision, slab geometries, the undeformed crystal, the splitting orders,
agreement with the 2D march when Ny = 1, the paper's 22 x 4267 x 1842 grid
on a sampled slice, and the calls a 3D plan refuses.

Tolerances as for the 2D march: FP64 1e-12 + 1e-14 Nz, the FP32-storage
modes 1e-5 (relL2 over both fields and per field, elementwise maximum,
phase)."""

import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.metrics import report, within

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def tol(prec, Nz):
    return 1e-12 + 1e-14 * Nz if prec == "fp64" else 1e-5


def gpu3(w, prec, workspace=False, order=1):
    from paper_2201_08500_amd import Plan3D
    p = Plan3D.from_workload(w, precision=prec, split_order=order)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = None if w.u is None else torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    ws = None
    if workspace:
        ws = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
    a, b = p.propagate(E0, u, workspace=ws)
    torch.cuda.synchronize()
    return a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128)


def oracle3(w, prec, slices=None, order=1):
    ws = w if slices is None else w.subset(slices)
    E0 = ws.E0_in if prec == "fp64" else ws.E0_in.astype(np.complex64).astype(np.complex128)
    return O.march3d(O.Problem3D.from_workload(ws, split_order=order), E0, ws.u)


def check3(w, prec, workspace=False, order=1):
    a, b = gpu3(w, prec, workspace, order)
    ra, rb = oracle3(w, prec, order=order)
    r = report(a, b, ra, rb)
    print(f"\n{w.name} {prec}: {r}", flush=True)
    bad = within(r, tol(prec, w.Nz), phase_tol=None if prec == "fp64" else 1e-4)
    assert not bad, (bad, r)
    return r


@pytest.mark.parametrize("prec", ["fp64", "fp32s", "fp32"])
@pytest.mark.parametrize("Nx,Ny", [
    (60, 6),       # Bluestein, L = 128
    (100, 5),      # Bluestein, odd Ny
    (251, 4),      # prime length, L = 512
    (32, 3),       # power of two below 64: Bluestein on L = 64
    (64, 8),       # direct transform
    (256, 1),      # one row
    (1000, 2),     # Bluestein, L = 2048
])
def test_3d_parity(Nx, Ny, prec):
    w = W.small3d(Nx=Nx, Ny=Ny, Nz=17, Nomega=2, seed=Nx + Ny)
    check3(w, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("Nx,Ny", [(2, 2), (3, 1), (5, 3)])
def test_3d_smallest_grids(Nx, Ny, prec):
    """The smallest transform lengths (Nx = 2, 3, 5 on L = 64) and Ny = 1."""
    check3(W.small3d(Nx=Nx, Ny=Ny, Nz=7, Nomega=2, seed=Nx), prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("Nx,Ny", [(60, 5), (256, 4), (3000, 2), (4267, 2)])
def test_3d_splitting_orders(Nx, Ny, order, prec):
    """Second- and fourth-order splitting (Eq. split-op) on the 3D grid:
    Bluestein, direct and four-step rows (Nx = 3000: L = 8192; Nx = 4267:
    L = 9216); order 4 uses two row-table sets (A lengths t dz and
    (1 - 2t) dz)."""
    check3(W.small3d(Nx=Nx, Ny=Ny, Nz=9, Nomega=2, seed=Nx + order), prec, order=order)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_3d_largest_ny_and_workspace_path(prec):
    w = W.small3d(Nx=90, Ny=32, Nz=11, Nomega=2, seed=7)
    check3(w, prec, workspace=True)


@pytest.mark.parametrize("slab", [
    dict(x_front=-1.0, thickness=math.inf),     # crystal everywhere
    dict(x_front=1.0, thickness=1.0),           # no crystal
    dict(x_front=-5e-6, thickness=8e-6),        # thin slab
])
def test_3d_slab_geometries(slab):
    w = W.small3d(Nx=72, Ny=4, Nz=13, Nomega=2, seed=3, **slab)
    check3(w, "fp64")


def test_3d_undeformed_and_long_rows():
    w = W.small3d(Nx=2048, Ny=3, Nz=9, Nomega=1, seed=5, deformed=False)
    check3(w, "fp64")
    w = W.small3d(Nx=3000, Ny=2, Nz=7, Nomega=1, seed=6)     # Bluestein, L = 8192
    check3(w, "fp64")
    check3(w, "fp32s")


@pytest.mark.parametrize("prec", ["fp64", "fp32s", "fp32"])
def test_3d_four_step_rows(prec):
    """Rows of 8192 and 16384 samples run in the four-step row kernel, whose
    tables are stored in its bin order: a power of two Nx = 8192 (L = Nx)
    and, where LDS allows (not FP64), Nx = 5000 (L = 16384)."""
    check3(W.small3d(Nx=8192, Ny=2, Nz=6, Nomega=1, seed=8), prec)
    if prec != "fp64":
        check3(W.small3d(Nx=5000, Ny=3, Nz=5, Nomega=2, seed=9), prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32s", "fp32"])
@pytest.mark.parametrize("Nx", [2049, 2304, 4097, 4267, 4608])
def test_3d_radix9_rows(Nx, prec):
    """2048 < Nx <= 2304 and 4096 < Nx <= 4608 run on rows of 9 M samples
    (L = 4608, 9216: nine wavefronts of M-point transforms and a radix-9
    step whose columns are read from and written to HBM directly), both
    ends of each range; FP64 rows of these lengths fit in LDS."""
    check3(W.small3d(Nx=Nx, Ny=3, Nz=5, Nomega=2, seed=Nx), prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("Nx,L", [(2048, 2048), (2305, 8192), (4096, 4096), (4609, 16384)])
def test_3d_row_length_boundaries(Nx, L, prec):
    """Either side of the lengths 9 M: 2305 and 4609 are the smallest Nx
    past 4608 and 9216 (next power of two), 2048 and 4096 are transformed
    directly.  FP64 rows of 16384 do not fit in LDS and are refused."""
    from paper_2201_08500_amd import BpmError
    w = W.small3d(Nx=Nx, Ny=2, Nz=5, Nomega=1, seed=Nx + 7)
    if prec == "fp64" and L > 9216:
        with pytest.raises(BpmError, match="FP64"):
            gpu3(w, prec)
        return
    check3(w, prec)


@pytest.mark.parametrize("order", [1, 2, 4])
def test_3d_one_row_matches_the_2d_march(order):
    """Ny = 1 on a power-of-two x grid: the 3D kernels and the 2D march
    compute the same problem (different transforms, so to rounding), for
    every splitting order."""
    from paper_2201_08500_amd import Plan
    w3 = W.small3d(Nx=512, Ny=1, Nz=40, Nomega=3, seed=12)
    a3, b3 = gpu3(w3, "fp64", order=order)
    p2 = Plan(w3.Nx, w3.dx, w3.dz, w3.Nz, w3.chi0, w3.chih, w3.chihbar, w3.theta_B,
              w3.lam, w3.Nomega, precision="fp64", x_front=w3.x_front,
              thickness=w3.thickness, delta=w3.delta, split_order=order)
    E0 = torch.from_numpy(np.ascontiguousarray(w3.E0_in[:, 0, :])).cuda()
    u = torch.from_numpy(np.ascontiguousarray(w3.u[:, 0, :])).cuda()
    a2, b2 = p2.propagate(E0, u)
    torch.cuda.synchronize()
    r = report(a3[:, 0, :], b3[:, 0, :], a2.cpu().numpy(), b2.cpu().numpy())
    assert not within(r, 1e-12 + 1e-14 * w3.Nz), r


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("Nx", [90, 4267])
def test_3d_general_mask(Nx, prec):
    """A crystal mask Pi(x, y, z) that changes with y and z (a wedge whose
    front moves with y, a hole in a few steps), with Strang splitting,
    against the oracle with the same mask."""
    from paper_2201_08500_amd import Plan3D
    w = W.small3d(Nx=Nx, Ny=6, Nz=14, Nomega=2, seed=31)
    x = (np.arange(w.Nx) - w.Nx // 2) * w.dx
    mask = np.zeros((w.Nz, w.Ny, w.Nx), dtype=bool)
    for n in range(w.Nz):
        for i in range(w.Ny):
            mask[n, i] = x >= (-6 + 2 * i - 0.5 * n) * 1e-6
    mask[5:8, :, ::7] = False
    p = Plan3D.from_workload(w, precision=prec, split_order=2, mask=mask)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    a, b = p.propagate(E0, u)
    torch.cuda.synchronize()
    E0r = w.E0_in if prec == "fp64" else w.E0_in.astype(np.complex64).astype(np.complex128)
    ra, rb = O.march3d(O.Problem3D.from_workload(w, split_order=2, mask=mask), E0r, w.u)
    r = report(a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128),
               ra, rb)
    assert not within(r, tol(prec, w.Nz), phase_tol=None if prec == "fp64" else 1e-4), r


@pytest.mark.parametrize("order,Nx", [(1, 100), (2, 100), (4, 100), (2, 4267)])
def test_3d_segments_chain_bitwise_fp64(order, Nx):
    """bpm_deformation_table, bpm_march and bpm_march_segment on a 3D plan:
    three segments chained through their outputs (the last in place) equal
    the whole march bitwise in FP64, and a segment resumed from a checkpoint
    of both envelopes matches the oracle started from that checkpoint."""
    from paper_2201_08500_amd import Plan3D
    w = W.small3d(Nx=Nx, Ny=5, Nz=12, Nomega=2, seed=40 + order)
    p = Plan3D.from_workload(w, precision="fp64", split_order=order)
    E0 = torch.from_numpy(w.E0_in).cuda()
    u = torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    ws = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
    p.deformation_table(u, ws)
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    p.march(E0, ws, a, b)
    a1, b1 = torch.empty_like(E0), torch.empty_like(E0)
    p.march_segment(E0, None, ws, 0, 5, a1, b1)
    a2, b2 = torch.empty_like(E0), torch.empty_like(E0)
    p.march_segment(a1, b1, ws, 5, 4, a2, b2)
    p.march_segment(a2, b2, ws, 9, 3, a2, b2)
    torch.cuda.synchronize()
    assert torch.equal(a2, a) and torch.equal(b2, b)
    # the whole march against the oracle, and the resumed part against the
    # oracle started at step 5 from the first segment's output
    r = report(a.cpu().numpy(), b.cpu().numpy(), *oracle3(w, "fp64", order=order))
    assert not within(r, tol("fp64", w.Nz)), r
    ra, rb = O.march3d(O.Problem3D.from_workload(w, split_order=order),
                       a1.cpu().numpy(), w.u[5:], n_steps=7, Eh_in=b1.cpu().numpy())
    r = report(a2.cpu().numpy(), b2.cpu().numpy(), ra, rb)
    assert not within(r, tol("fp64", 7)), r


def test_3d_segments_fp32s_within_rounding():
    """FP32 storage: each segment boundary stores the state in FP32, so the
    chained march differs from the whole one at the mode's rounding level."""
    from paper_2201_08500_amd import Plan3D
    w = W.small3d(Nx=3000, Ny=2, Nz=10, Nomega=1, seed=50)
    p = Plan3D.from_workload(w, precision="fp32s", split_order=2)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    ws = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
    p.deformation_table(u, ws)
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    p.march(E0, ws, a, b)
    c, d = torch.empty_like(E0), torch.empty_like(E0)
    p.march_segment(E0, None, ws, 0, 6, c, d)
    p.march_segment(c, d, ws, 6, 4, c, d)
    torch.cuda.synchronize()
    r = report(c.cpu().numpy().astype(np.complex128), d.cpu().numpy().astype(np.complex128),
               a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128))
    assert not within(r, 1e-6), r


@pytest.mark.parametrize("prec", ["fp32s", "fp64", "fp32"])
def test_3d_paper_grid_sampled_slice(prec):
    """The grid of the paper's finite-element example, 22 x 4267 x 1842
    (rows of L = 9216), two slices; the oracle recomputes one of them."""
    w = W.heat_bump_3d(Nomega=2)
    a, b = gpu3(w, prec)
    ra, rb = oracle3(w, prec, slices=[1])
    r = report(a[1:2], b[1:2], ra, rb)
    print(f"\n{w.name} {prec} slice 1: {r}", flush=True)
    assert not within(r, tol(prec, w.Nz), phase_tol=None if prec == "fp64" else 1e-4), r


def test_3d_plan_refuses_what_it_does_not_support():
    from paper_2201_08500_amd import BpmError, Job, Plan3D, propagate_batch
    w = W.small3d(Nx=60, Ny=4, Nz=5, Nomega=1, seed=1)
    p = Plan3D.from_workload(w, precision="fp32s")
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = torch.from_numpy(w.u).cuda()
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    for call in (lambda: p.propagate_noalloc(E0, u, a, b),
                 lambda: propagate_batch([Job(p, E0, u)])):
        with pytest.raises(BpmError):
            call()
    # FP64 rows beyond the LDS: Nx = 5000 needs L = 16384
    big = W.small3d(Nx=5000, Ny=1, Nz=2, Nomega=1, seed=2)
    pb = Plan3D.from_workload(big, precision="fp64")
    Eb = torch.from_numpy(big.E0_in).cuda()
    with pytest.raises(BpmError, match="FP64"):
        pb.propagate(Eb, torch.from_numpy(big.u).cuda())
