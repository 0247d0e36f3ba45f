"""GPU parity of the two-halves rotate-on-write pass of length 2048
(DFT3D_OPT_HALVES): the radix-2 split x[n] +- x[n + 1024], the difference
twiddled by w_2048^n, and each half through the 1024-point stages in one
16-pencil LDS tile, the even outputs first.  Ordinary and streaming
accesses, forward and inverse, element by element against the FP64 oracle,
with ragged last tiles and grids of more tiles than resident workgroups; the
pass is the same whatever the persistent option says (it has one form)."""
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


def execute(x, inverse=False, **kw):
    xt = torch.from_numpy(x).cuda()
    y = torch.empty_like(xt)
    p = dft3d.Plan(x.shape, "pencil", **kw)
    p.execute(xt, y, inverse=inverse)
    torch.cuda.synchronize()
    p.close()
    return y.cpu().numpy()


def reference(x, sign):
    """FP64 oracle: O2 where every axis is a power of two, else O1."""
    pow2 = all(n & (n - 1) == 0 for n in x.shape)
    return oracle.dft3d(x.astype(np.complex128), sign, "fft" if pow2 else "direct")


def halves_passes(shape, **kw):
    d = dft3d.describe(shape, "pencil", **kw)
    return [p for p in d["passes"] if p["halves"]]


# (shape, pencils of the 2048 pass): fewer than one tile, a ragged second
# tile, 2048 as the middle and the first axis
SHAPES = [(2048, 3, 5), (2048, 17, 2), (2, 2048, 40), (33, 2, 2048)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("nontemporal", [0, 1])
def test_halves_element_by_element(shape, persistent, nontemporal):
    say("case halves", shape, "persistent", persistent, "nontemporal", nontemporal)
    kw = dict(persistent=persistent, nontemporal=nontemporal)
    hp = halves_passes(shape, **kw)
    assert len(hp) == 1 and hp[0]["tile"] == 16 and hp[0]["persistent"] == 0
    assert hp[0]["nontemporal"] == nontemporal and hp[0]["radices"] == [2, 32, 32]
    x = inputs.uniform_c64(shape, 71)
    for sign, inv in ((-1, False), (1, True)):
        y = execute(x, inverse=inv, **kw)
        ref = reference(x, sign)
        rel, worst = oracle.compare(y, ref)
        say("  ", sign, rel, worst)
        assert rel <= oracle.tol(x.size), (shape, sign, rel)
        assert worst <= 10 * oracle.tol(x.size), (shape, sign, worst)


def test_halves_off_keeps_the_whole_length_kernel():
    shape = (2048, 17, 2)
    assert not halves_passes(shape, halves=0)
    assert not halves_passes(shape, tile=8)
    x = inputs.uniform_c64(shape, 72)
    ref = reference(x, -1)
    for kw in ({"halves": 0}, {"halves": 1}):
        rel, worst = oracle.compare(execute(x, **kw), ref)
        say("case halves option", kw, rel, worst)
        assert rel <= oracle.tol(x.size) and worst <= 10 * oracle.tol(x.size), kw


@pytest.mark.parametrize("shape", [(2048, 64, 128), (2048, 65, 67)])
@pytest.mark.parametrize("persistent", [0, 1])
def test_halves_many_tiles_per_workgroup(shape, persistent):
    """More tiles than resident workgroups (512 tiles; 273 with a last tile
    of 3 pencils), with the other passes in both forms."""
    say("case halves many tiles", shape, "persistent", persistent)
    kw = dict(persistent=persistent, nontemporal=1)
    assert halves_passes(shape, **kw)[0]["pencils"] == shape[1] * shape[2]
    x = inputs.uniform_c64(shape, 73)
    for sign, inv in ((-1, False), (1, True)):
        y = execute(x, inverse=inv, **kw)
        rel, worst = oracle.compare(y, reference(x, sign))
        say("  ", sign, rel, worst)
        assert rel <= oracle.tol(x.size), (sign, rel)
        assert worst <= 10 * oracle.tol(x.size), (sign, worst)
