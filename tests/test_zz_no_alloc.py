"""The allocation-free apply (rst_apply_h_noalloc) against rst_apply_h, through
the C ABI: the same operator on the same columns, two calls in a row, the second
with fewer columns; its size limit; and no device memory taken by its calls."""
import numpy as np
import pytest

from paper_2208_02783_amd import rst
from paper_2208_02783_amd import workloads as wl
from tests.gpu_util import make_ctx, torch_cuda

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 16 << 20


def _pair(torch, ctx_ref, ctx_na, e, x, prec):
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, float("nan"))
    torch.cuda.synchronize()
    ctx_ref.rst_apply_h(e, x.data_ptr(), y_ref.data_ptr(), x.shape[1], prec)
    ctx_na.rst_apply_h_noalloc(e, x.data_ptr(), y_na.data_ptr(), x.shape[1], prec)
    return y_ref, y_na


@pytest.mark.parametrize("prec", [rst.RST_FP64, rst.RST_FP32_REFINE])
def test_noalloc_apply_equals_apply_twice(prec):
    """Config 2 (17x17x170, 360 projectors): 96 columns, then 23; the outputs equal
    rst_apply_h's (same kernels: bitwise, within the apply bar 1e-13 max|y| at
    least), and the second call's smaller projection block does not see the
    first call's leftovers."""
    torch = torch_cuda()
    p = wl.config(2)
    k = p.kpts[3]
    ctx_ref = make_ctx(torch, p, k)
    ctx_na = make_ctx(torch, p, k)
    dt = torch.complex128 if prec == rst.RST_FP64 else torch.complex64
    g = torch.Generator(device="cuda").manual_seed(21)
    xs = [torch.randn((p.n, nc), dtype=torch.complex128, device="cuda", generator=g).to(dt) for nc in (96, 23)]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    outs = [_pair(torch, ctx_ref, ctx_na, float(p.energies[200 + 50 * i]), x, prec) for i, x in enumerate(xs)]
    torch.cuda.synchronize()
    for y_ref, y_na in outs:
        assert torch.isfinite(torch.view_as_real(y_na)).all()
        d = (torch.max(torch.abs(y_na - y_ref)) / torch.max(torch.abs(y_ref))).item()
        assert d <= 1e-13, d
    # the no-allocation context took no device memory for its two calls (the reference
    # context grew its projection buffer, so only check the no-allocation context alone)
    y = torch.empty_like(xs[0])
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    ctx_na.rst_apply_h_noalloc(0.3, xs[0].data_ptr(), y.data_ptr(), xs[0].shape[1], prec)
    ctx_na.rst_apply_h_noalloc(0.4, xs[1].data_ptr(), y.data_ptr(), xs[1].shape[1], prec)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free1
    assert free0 > 0


def test_noalloc_apply_limit_and_errors():
    """Beyond the scratch size the call is refused (RST_EINVAL) and writes nothing;
    without projectors there is no limit; zero columns is a no-op."""
    torch = torch_cuda()
    p = wl.config(2, tiny=True)  # 216 projectors
    ctx = make_ctx(torch, p, p.kpts[0])
    cmax = SCRATCH_BYTES // (16 * p.proj.nproj)
    x = torch.zeros((p.n, cmax + 1), dtype=torch.complex128, device="cuda")
    y = torch.full_like(x, 7.0)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_apply_h_noalloc(0.5, x.data_ptr(), y.data_ptr(), cmax + 1, rst.RST_FP64)
    assert ei.value.status == rst.RST_EINVAL
    torch.cuda.synchronize()
    assert torch.all(y == 7.0)
    ctx.rst_apply_h_noalloc(0.5, x.data_ptr(), y.data_ptr(), cmax, rst.RST_FP64)  # n x cmax in the buffer's head
    torch.cuda.synchronize()
    assert torch.all(y.reshape(-1)[:p.n * cmax] == 0.0)
    ctx.rst_apply_h_noalloc(0.5, x.data_ptr(), y.data_ptr(), 0, rst.RST_FP64)
    with pytest.raises(rst.RstError) as ei:
        ctx.rst_apply_h_noalloc(0.5, x.data_ptr(), x.data_ptr(), 4, rst.RST_FP64)
    assert ei.value.status == rst.RST_EINVAL
    p1 = wl.config(1)  # no projectors: no scratch needed at any width
    c1 = make_ctx(torch, p1, (0.0, 0.0))
    x1 = torch.ones((p1.n, 3000), dtype=torch.complex128, device="cuda")
    y1 = torch.empty_like(x1)
    y2 = torch.empty_like(x1)
    c1.rst_apply_h_noalloc(0.5, x1.data_ptr(), y1.data_ptr(), 3000, rst.RST_FP64)
    c1.rst_apply_h(0.5, x1.data_ptr(), y2.data_ptr(), 3000, rst.RST_FP64)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
