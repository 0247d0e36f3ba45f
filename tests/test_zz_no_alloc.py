"""GPU test of dft3d_execute_noalloc, the entry point that allocates
nothing: its workspace is the library's static per-device array.  Its output
must equal dft3d_execute's on the same plan bitwise (same kernels, same
arithmetic), on two calls in a row with the second one smaller, and match the
FP64 oracle within the stated tolerance."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAX_WS = 128 << 20  # DFT3D_NOALLOC_MAX_WORKSPACE


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def say(*a):
    print(*a, flush=True)


def run_noalloc(plan, x, out, sign):
    st = dft3d.lib().dft3d_execute_noalloc(
        plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
        sign, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("schedule", ["pencil", "volumetric"])
def test_noalloc_matches_execute_two_calls(schedule):
    # first call: the largest workspace the entry point serves (256^3 points,
    # 128 MiB); second call: a smaller ragged shape on another plan
    for shape, seed in (((256, 256, 256), 11), ((48, 40, 24) if schedule == "pencil"
                                                 else (64, 32, 128), 12)):
        say("case noalloc", schedule, shape)
        x_h = inputs.uniform_c64(shape, seed)
        x = torch.from_numpy(x_h).cuda()
        p = dft3d.Plan(shape, schedule)
        need = p.workspace_size()
        assert 0 < need <= MAX_WS
        for sign in (-1, 1):
            ref = torch.empty_like(x)
            p.execute(x, ref, inverse=(sign == 1))
            got = torch.full_like(x, float("nan"))
            assert run_noalloc(p, x, got, sign) == dft3d.OK
            torch.cuda.synchronize()
            assert torch.equal(got.view(torch.float32), ref.view(torch.float32)), (shape, sign)
            if x_h.size <= 1 << 16:
                o = oracle.dft3d(x_h.astype(np.complex128), sign, "direct")
                err = oracle.rel_l2(got.cpu().numpy(), o)
                assert err <= oracle.tol(x_h.size), (shape, sign, err)
        p.close()


def test_noalloc_rejects_oversized_workspace_and_takes_slab():
    # 512 x 256 x 256 pencil needs 256 MiB of workspace: refused before any
    # launch; the slab schedule needs none and runs at that size
    shape = (512, 256, 256)
    p = dft3d.Plan(shape, "pencil")
    assert p.workspace_size() > MAX_WS
    x = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    assert run_noalloc(p, x, y, -1) == dft3d.ERR_WORKSPACE_TOO_SMALL
    p.close()
    x_h = inputs.uniform_c64(shape, 13)
    x = torch.from_numpy(x_h).cuda()
    q = dft3d.Plan(shape, "slab")
    assert q.workspace_size() == 0
    ref = torch.empty_like(x)
    q.execute(x, ref)
    assert run_noalloc(q, x, y, -1) == dft3d.OK
    torch.cuda.synchronize()
    assert torch.equal(y.view(torch.float32), ref.view(torch.float32))
    # bad arguments are refused before anything is enqueued
    assert run_noalloc(q, x, x, -1) == dft3d.ERR_INVALID_ARG
    assert run_noalloc(q, x, y, 0) == dft3d.ERR_INVALID_ARG
    # the Python binding's method goes through the same entry point
    y.zero_()
    q.execute_noalloc(x, y)
    torch.cuda.synchronize()
    assert torch.equal(y.view(torch.float32), ref.view(torch.float32))
    q.close()
