"""GPU tests of the move-only plans (DFT3D_OPT_MOVE_ONLY): the schedules'
data movement without the radix stages (mode 1), whose output must equal,
bit for bit, the permutation of the input the CPU model of the pass maps
gives (tests/test_plan_model.py: the pass's load and store maps with every
pencil permuted by the Stockham stage maps of its radices), and plain copies
(mode 2), whose output is the input."""
import numpy as np
import pytest

from paper_1904_10119_amd import dft3d, inputs
from test_plan_model import run_move_model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("shape", [(16, 32, 64), (64, 64, 64), (128, 4, 256), (2048, 2, 8),
                                   (256, 256, 256)])
@pytest.mark.parametrize("schedule", ["pencil", "slab", "volumetric"])
@pytest.mark.parametrize("mode", [1, 2])
def test_move_only_output_is_the_modelled_permutation(shape, schedule, mode):
    print("case move-only", shape, schedule, mode, flush=True)
    x = inputs.uniform_c64(shape, 61)
    d = dft3d.describe(shape, schedule, move_only=mode)
    xt = torch.from_numpy(x).cuda()
    p = dft3d.Plan(shape, schedule, move_only=mode)
    for inverse, sign in ((False, -1), (True, 1)):
        y = torch.full_like(xt, float("nan"))
        p.execute(xt, y, inverse=inverse)
        torch.cuda.synchronize()
        want = run_move_model(x, d, sign)
        assert np.array_equal(bits(y.cpu().numpy()), bits(want)), (shape, schedule, mode, sign)
    p.close()


def test_move_only_streaming_persistent_kernels():
    """Shapes of 512 MiB and more: (1024, 1024, 64) on the pencil schedule
    in its default form (the cycled order's one-tile kernels, which the
    1024^3 breakdown times) and with streaming forced (the persistent
    streaming kernels), on the slab schedule with the whole-length kernels
    (persistent, streaming) and with the strided passes as two halves, every
    element against the model."""
    shape = (1024, 1024, 64)
    x = inputs.uniform_c64(shape, 62)
    xt = torch.from_numpy(x).cuda()
    for schedule, halves, nt in (("pencil", 0, -1), ("pencil", 0, 1), ("slab", 0, -1),
                                 ("slab", 1, -1)):
        print("case move-only streaming", shape, schedule, "halves", halves, "nt", nt,
              flush=True)
        opts = {"nontemporal": nt} if nt >= 0 else {}
        d = dft3d.describe(shape, schedule, move_only=1, halves=halves, **opts)
        if halves:
            assert sum(p["halves"] for p in d["passes"]) == 2
        elif schedule == "pencil" and nt < 0:
            assert all("cyc" in p["label"].split() and not p["persistent"] for p in d["passes"])
        else:
            assert any(p["persistent"] and p["nontemporal"] == 1 for p in d["passes"])
        y = torch.empty_like(xt)
        p = dft3d.Plan(shape, schedule, move_only=1, halves=halves, **opts)
        p.execute(xt, y)
        torch.cuda.synchronize()
        assert np.array_equal(bits(y.cpu().numpy()), bits(run_move_model(x, d)))
        p.close()
