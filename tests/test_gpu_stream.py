"""The streamed last order (options.stream_last): solving the last order in
slices gives the result of the one-call run (lists, energies and increments
bitwise, the gradient up to the order of the device's atomic adds), and the
slices keep the contract (each tuple once, close only when complete)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(8 << 30)


@pytest.mark.parametrize("gradient", [0, 1])
def test_streamed_order_equals_one_call(ws, gradient):
    P = synth.config_plain(0)
    opts = dict(max_order=4, gradient=gradient)
    ref_ctx = M.Context.from_problem(P, device=0, **opts)
    ref, ref_h = ref_ctx.run(ws, keep=True)
    ctx = M.Context.from_problem(P, device=0, stream_last=1, **opts)
    part, h = ctx.run(ws, keep=True)
    o4 = part.orders[-1]
    assert o4.k == 4 and (o4.status == M.TUPLE_PENDING).all() and np.isnan(o4.eps).all()
    n4 = len(o4.tuples)
    assert n4 == 70
    with pytest.raises(M.MBEFCIError) as e:
        ctx.backward(h, ws)                       # order still open
    assert e.value.code == -5
    stride = 3
    for first in range(stride):
        cnt = len(range(first, n4, stride))
        if first == 2:
            with pytest.raises(M.MBEFCIError) as e:
                ctx.order_close(h)                # not every tuple solved
            assert e.value.code == -5
        ctx.order_solve(h, first, stride, cnt, ws)
    with pytest.raises(M.MBEFCIError) as e:
        ctx.order_solve(h, 0, 1, 1, ws)           # solved already
    assert e.value.code == -1
    res = ctx.order_close(h)
    for a, b in zip(res.orders, ref.orders):
        assert np.array_equal(a.tuples, b.tuples)
        assert np.array_equal(a.eps, b.eps) and np.array_equal(a.dinc, b.dinc)
        assert a.order_sum == b.order_sum
        assert (a.status == 0).all()
    assert res.total == ref.total
    if gradient:
        gh, ge = ctx.backward(h, ws)
        rh, re_ = ref_ctx.backward(ref_h, ws)
        print(f"streamed vs one-call gradient: {np.abs(gh - rh).max():.1e} {np.abs(ge - re_).max():.1e}")
        assert np.abs(gh - rh).max() <= 1e-12 and np.abs(ge - re_).max() <= 1e-12
