"""GPU parity of the wide one-tile split-precision pass (rotate-on-write,
length 2048, 8 pencils per workgroup where the default tile has 4; the
default one-tile form at that length): every split and single-term
precision, both leaf lengths, forward and inverse, ragged and multi-tile
grids, element by element against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPLIT = ["bf16x6", "bf16x9", "fp16x3"]
SINGLE = {"bf16x1": 2e-2, "fp16x1": 3e-3}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def say(*a):
    print(*a, flush=True)


def execute(x, inverse=False, **kw):
    xt = torch.from_numpy(x).cuda()
    y = torch.empty_like(xt)
    p = dft3d.Plan(x.shape, "pencil", **kw)
    p.execute(xt, y, inverse=inverse)
    torch.cuda.synchronize()
    p.close()
    return y.cpu().numpy()


@pytest.mark.parametrize("precision", SPLIT + list(SINGLE))
@pytest.mark.parametrize("leaf", [16, 32])
@pytest.mark.parametrize("tile", [0, 8])
@pytest.mark.parametrize("others", [(2, 2), (8, 16)])
def test_wide_element_by_element(precision, leaf, tile, others):
    n = 2048
    shape = others + (n,)
    kw = dict(precision=precision, mfma_leaf=leaf, tile=tile, persistent=0)
    say("case mfma wide", precision, leaf, shape, "tile", tile)
    d = dft3d.describe(shape, "pencil", **kw)
    p = [q for q in d["passes"] if q["n"] == n]
    assert len(p) == 1 and p[0]["tile"] == 8 and p[0]["threads"] == 1024
    assert p[0]["mfma_leaf"] == leaf and p[0]["persistent"] == 0
    x = inputs.uniform_c64(shape, 400 + n % 97 + leaf)
    for sign, inv in ((-1, False), (1, True)):
        y = execute(x, inverse=inv, **kw)
        ref = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        rel, worst = oracle.compare(y, ref)
        say("  ", sign, rel, worst)
        if precision in SPLIT:
            assert rel <= oracle.tol(x.size), (precision, shape, sign, rel)
            assert worst <= 10 * oracle.tol(x.size), (precision, shape, sign, worst)
        else:
            assert rel <= SINGLE[precision], (precision, shape, sign, rel)


def test_default_tile_and_other_tiles():
    """Length 2048 takes the wide form by default in split precision; tile 4
    or the persistent form ask for the default-tile kernels."""
    for prec in SPLIT:
        d = dft3d.describe((2, 2, 2048), "pencil", precision=prec)
        assert [(q["tile"], q["persistent"]) for q in d["passes"] if q["n"] == 2048] == [(8, 0)]
        d = dft3d.describe((2, 2, 2048), "pencil", precision=prec, tile=4)
        assert [q["tile"] for q in d["passes"] if q["n"] == 2048] == [4]
        d = dft3d.describe((2, 2, 2048), "pencil", precision=prec, nontemporal=1)
        assert [(q["tile"], q["persistent"]) for q in d["passes"] if q["n"] == 2048] == [(4, 1)]
