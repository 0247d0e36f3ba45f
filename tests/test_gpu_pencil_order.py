"""GPU parity of the pencil schedule's intermediate orders
(DFT3D_OPT_PENCIL_ORDER): the rotation, the swap of the two fastest axes
and the cycle, in FP32 (whole-length, halves and persistent kernels) and
split precision (one-tile, wide and persistent matrix-core kernels), forward
and inverse, element by element against the FP64 oracle, with ragged tiles
and every axis in every position."""
import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def say(*a):
    print(*a, flush=True)


SHAPES = [(16, 32, 64), (2, 1024, 8), (2048, 4, 2), (8, 2, 2048), (64, 64, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("precision", ["fp32", "bf16x6", "fp16x3"])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("persistent", [0, 1])
def test_order_element_by_element(shape, precision, order, persistent):
    say("case pencil order", shape, precision, order, "persistent", persistent)
    kw = dict(precision=precision, pencil_order=order, persistent=persistent)
    if persistent:
        kw["nontemporal"] = 1  # the persistent forms at these sizes
    d = dft3d.describe(shape, "pencil", **kw)
    tag = {1: "swap", 2: "cyc"}[order]
    assert d["passes"][0]["label"].endswith(tag)
    x = inputs.uniform_c64(shape, 90 + order)
    xt = torch.from_numpy(x).cuda()
    p = dft3d.Plan(shape, "pencil", **kw)
    for sign, inv in ((-1, False), (1, True)):
        y = torch.empty_like(xt)
        p.execute(xt, y, inverse=inv)
        torch.cuda.synchronize()
        rel, worst = oracle.compare(y.cpu().numpy(), oracle.dft3d(x.astype(np.complex128), sign, "fft"))
        say("  ", sign, rel, worst)
        assert rel <= oracle.tol(x.size), (shape, precision, order, sign, rel)
        assert worst <= 10 * oracle.tol(x.size), (shape, precision, order, sign, worst)
    p.close()
