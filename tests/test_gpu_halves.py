"""GPU parity of the two-halves passes (DFT3D_OPT_HALVES): the radix-2
split x[n] +- x[n + N/2], the difference twiddled by w_N^n, and each half
through the N/2-point stages in one LDS tile of twice the pencils, the even
outputs first -- the rotate-on-write pass of length 2048 (16 pencils) and
the strided in-place passes of the slab schedule (2048: 16 pencils, 1024:
32).  Ordinary and streaming accesses, forward and
inverse, one tile per workgroup and persistent (the next tile's lower
halves loaded during the current tile's second half), element by element
against the FP64 oracle, with ragged last tiles and grids of more tiles than
resident workgroups."""
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


def execute(x, schedule="pencil", inverse=False, **kw):
    xt = torch.from_numpy(x).cuda()
    y = torch.empty_like(xt)
    p = dft3d.Plan(x.shape, schedule, **kw)
    p.execute(xt, y, inverse=inverse)
    torch.cuda.synchronize()
    p.close()
    return y.cpu().numpy()


def reference(x, sign):
    """FP64 oracle: O2 where every axis is a power of two, else O1."""
    pow2 = all(n & (n - 1) == 0 for n in x.shape)
    return oracle.dft3d(x.astype(np.complex128), sign, "fft" if pow2 else "direct")


# (schedule, shape, fused_plane option, the halves passes (n, load, store)):
# fewer pencils than one tile, a ragged last tile, every axis position
CASES = [
    ("pencil", (2048, 3, 5), 1, [(2048, "row", "col")]),
    ("pencil", (2048, 17, 2), 1, [(2048, "row", "col")]),
    ("pencil", (2, 2048, 40), 1, [(2048, "row", "col")]),
    ("pencil", (33, 2, 2048), 1, [(2048, "row", "col")]),
    ("slab", (1024, 1024, 2), 0, [(1024, "col", "col")] * 2),
    ("slab", (1024, 4, 2), 0, [(1024, "col", "col")]),
    ("slab", (1024, 2, 64), 0, [(1024, "col", "col")]),
    ("slab", (8, 1024, 16), 0, [(1024, "col", "col")]),
    ("slab", (2048, 4, 8), 0, [(2048, "col", "col")]),
    ("slab", (2048, 32, 2), 0, [(2048, "col", "col")]),
]


def halves_passes(shape, schedule="pencil", **kw):
    d = dft3d.describe(shape, schedule, **kw)
    return [p for p in d["passes"] if p["halves"]]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}")
@pytest.mark.parametrize("nontemporal", [0, 1])
@pytest.mark.parametrize("persistent", [0, 1])
def test_halves_element_by_element(case, nontemporal, persistent):
    schedule, shape, fused_plane, want = case
    say("case halves", schedule, shape, "nontemporal", nontemporal, "persistent", persistent)
    kw = dict(nontemporal=nontemporal, fused_plane=fused_plane, persistent=persistent)
    hp = halves_passes(shape, schedule, **kw)
    assert [(p["n"], p["load"], p["store"]) for p in hp] == want, hp
    for p in hp:
        # the strided 2048 pass has one tile per workgroup only
        pers = persistent and not (p["n"] == 2048 and p["load"] == "col")
        assert p["tile"] == 32768 // p["n"] and p["persistent"] == pers
        assert p["nontemporal"] == nontemporal and p["radices"][0] == 2
    x = inputs.uniform_c64(shape, 71)
    for sign, inv in ((-1, False), (1, True)):
        y = execute(x, schedule, inverse=inv, **kw)
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
        rel, worst = oracle.compare(execute(x, "pencil", **kw), ref)
        say("case halves option", kw, rel, worst)
        assert rel <= oracle.tol(x.size) and worst <= 10 * oracle.tol(x.size), kw


@pytest.mark.parametrize("shape", [(2048, 64, 128), (2048, 65, 67)])
@pytest.mark.parametrize("persistent", [0, 1])
def test_halves_many_tiles_per_workgroup(shape, persistent):
    """More tiles than resident workgroups (512 tiles; 273 with a last tile
    of 3 pencils): the persistent form walks several tiles per workgroup."""
    say("case halves many tiles", shape, "persistent", persistent)
    kw = dict(persistent=persistent, nontemporal=1)
    hp = halves_passes(shape, **kw)
    assert hp[0]["pencils"] == shape[1] * shape[2] and hp[0]["persistent"] == persistent
    x = inputs.uniform_c64(shape, 73)
    for sign, inv in ((-1, False), (1, True)):
        y = execute(x, "pencil", inverse=inv, **kw)
        rel, worst = oracle.compare(y, reference(x, sign))
        say("  ", sign, rel, worst)
        assert rel <= oracle.tol(x.size), (sign, rel)
        assert worst <= 10 * oracle.tol(x.size), (sign, worst)
