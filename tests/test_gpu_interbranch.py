"""The interbranch-scattering case of Section 3.2 on the GPU: the deformed
march at Nx = 4096 with a deformation phase whose gradient reaches half the
grid's Nyquist limit.  Parity with the oracle on the same inputs, and the
new branch's power against exp(-2 pi beta_c / |beta|) (the analytic value
the oracle pin checks, same protocol)."""

import math

import numpy as np
import pytest
import torch

import oracle as O
from test_oracle_interbranch import (B, CHI0, DX, DZ, LAM, NX, NZ, TH, THICK,
                                     W0, X0, chih_for)
from workloads.metrics import report, within

pytestmark = pytest.mark.gpu


def inputs(ratio):
    chih = chih_for(ratio)
    k0 = 2 * math.pi / LAM
    h = 2 * k0 * math.sin(TH)
    x = (np.arange(NX) - NX // 2) * DX
    th_i = TH - CHI0 / math.sin(2 * TH) + 6.0 * 2 * chih / math.sin(2 * TH)
    E0 = (np.exp(-((x - X0) / W0) ** 2)
          * np.exp(1j * (k0 * math.sin(th_i) - 0.5 * h) * x))[None, :]
    u = np.ascontiguousarray(np.broadcast_to(np.where(x >= 0, B * x ** 2, 0.0), (NZ, NX)))
    return chih, x, E0, u


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_interbranch_on_gpu(prec):
    from paper_2201_08500_amd import Plan
    ratio = 4.7326
    chih, x, E0, u = inputs(ratio)
    p = Plan(NX, DX, DZ, NZ, CHI0, -chih, -chih, TH, LAM, 1, precision=prec,
             x_front=0.0, thickness=THICK, delta=[0.0])
    a, b = p.propagate(torch.from_numpy(E0).to(p.field_dtype).cuda(),
                       torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    a = a.cpu().numpy().astype(np.complex128)
    b = b.cpu().numpy().astype(np.complex128)
    q = O.Problem(NX, DX, DZ, NZ, CHI0, -chih, -chih, TH, LAM, [0.0],
                  x_front=0.0, thickness=THICK)
    E_ref = E0 if prec == "fp64" else E0.astype(np.complex64).astype(np.complex128)
    ra, rb = O.march(q, E_ref, u)
    r = report(a, b, ra, rb)
    assert not within(r, 1e-12 + 1e-14 * NZ if prec == "fp64" else 1e-5), r
    T = np.sum(np.abs(a[0, x >= THICK]) ** 2) / np.sum(np.abs(E0) ** 2)
    assert abs(T / math.exp(-2 * math.pi / ratio) - 1) < 0.03, T
