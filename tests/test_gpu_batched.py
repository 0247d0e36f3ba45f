"""GPU tests of the batched form (dft3d_execute_batched): many 3D DFTs of
different shapes, one launch per pass level covering every problem, or the
whole batch in one persistent launch (DFT3D_OPT_BATCH_LAUNCH = 1: a device
ticket queue with per-item completion counters, replayed from a HIP graph
the library builds)."""
import os
import sys

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


def make_batch(shapes, seed):
    xs = [inputs.uniform_c64(s, seed + i) for i, s in enumerate(shapes)]
    return xs, [torch.from_numpy(x).cuda() for x in xs]


def check_against_oracle(xs, ys, sign):
    for x, y in zip(xs, ys):
        ref = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        err = oracle.rel_l2(y.cpu().numpy(), ref)
        assert err <= oracle.tol(x.size), (x.shape, sign, err)


@pytest.mark.parametrize("schedule", ["pencil", "slab", "auto"])
def test_batched_small_mixed_shapes(schedule):
    """One persistent launch for a batch of mixed shapes (including 1^3 and
    2^3): every result against the oracle and its single-plan execution."""
    shapes = [(32, 64, 128), (128, 32, 64), (64, 64, 64), (8, 16, 4), (2, 2, 2),
              (1, 1, 1), (32, 32, 32), (128, 128, 16)]
    say("case persistent batched", schedule, shapes)
    xs, xt = make_batch(shapes, 40)
    ys = dft3d.fftn_batched(xt, schedule=schedule, launch="persistent")
    torch.cuda.synchronize()
    check_against_oracle(xs, ys, -1)
    # each equals its single-plan execution to within the tolerance
    for x, y in zip(xt, ys):
        single = dft3d.fftn(x, schedule=schedule)
        torch.cuda.synchronize()
        assert oracle.rel_l2(y.cpu().numpy(), single.cpu().numpy()) <= oracle.tol(x.numel())


def test_batched_96_problems_replays_and_inverse():
    """The uneven 96-problem workload in one persistent launch: the first
    call builds the graph, later calls replay it (same buffers, new values),
    with eager work in between; then other output buffers and the inverse."""
    shapes = inputs.batch_shapes(96, 104)
    say("case persistent batched 96", len(shapes))
    xs, xt = make_batch(shapes, 500)
    outs = [torch.empty_like(x) for x in xt]
    for rep in range(3):
        dft3d.fftn_batched(xt, outs=outs, launch="persistent")
        torch.cuda.synchronize()
        # eager work between replays, through the same plans
        eager = [dft3d.fftn(x) for x in xt[:4]]
        torch.cuda.synchronize()
        for i in range(0, 96, 7):
            ref = oracle.dft3d(xs[i].astype(np.complex128), -1, "fft")
            assert oracle.rel_l2(outs[i].cpu().numpy(), ref) <= oracle.tol(xs[i].size), (rep, i)
        for e, o in zip(eager, outs[:4]):
            assert oracle.rel_l2(o.cpu().numpy(), e.cpu().numpy()) <= oracle.tol(o.numel())
        # new inputs for the next replay (same plans, same buffers rewritten)
        for i in range(96):
            xs[i] = inputs.uniform_c64(shapes[i], 900 + 96 * rep + i)
            xt[i].copy_(torch.from_numpy(xs[i]))
    # different output buffers: pointers refreshed without a new graph
    outs2 = dft3d.fftn_batched(xt, inverse=True, launch="persistent")
    torch.cuda.synchronize()
    for i in range(0, 96, 11):
        ref = oracle.dft3d(xs[i].astype(np.complex128), +1, "fft")
        assert oracle.rel_l2(outs2[i].cpu().numpy(), ref) <= oracle.tol(xs[i].size)


def test_batched_long_axes_fall_back_plan_by_plan():
    shapes = [(1024, 4, 8), (16, 16, 16)]
    xs, xt = make_batch(shapes, 60)
    ys = dft3d.fftn_batched(xt)
    torch.cuda.synchronize()
    check_against_oracle(xs, ys, -1)


def test_batched_count_zero_and_bad_args():
    L = dft3d.lib()
    assert L.dft3d_execute_batched(None, None, None, 0, -1, None) == dft3d.OK
    p = dft3d.Plan((4, 4, 4), "pencil")
    x = torch.zeros((4, 4, 4), dtype=torch.complex64, device="cuda")
    import ctypes
    arr = ctypes.c_void_p * 1
    st = L.dft3d_execute_batched(arr(p.handle.value), arr(x.data_ptr()),
                                 arr(x.data_ptr()), 1, -1, None)
    assert st == dft3d.ERR_INVALID_ARG  # in == out
    p.close()


def test_bounded_wait_reports_instead_of_hanging(monkeypatch):
    """A spin limit of one poll forces the persistent kernel's dependency
    waits to run out: the launch must still finish, and with the check hook
    the call reports the condition as an error.  A later batch on other
    plans (default limit) is correct again."""
    monkeypatch.setenv("DFT3D_BATCH_SPIN_LIMIT", "1")
    monkeypatch.setenv("DFT3D_BATCH_CHECK", "1")
    shapes = inputs.batch_shapes(96, 7)
    say("case bounded wait", len(shapes))
    plans = [dft3d.Plan(s, "pencil", batch_launch=1) for s in shapes]  # fresh descriptors
    xt = [torch.zeros(s, dtype=torch.complex64, device="cuda") for s in shapes]
    outs = [torch.empty_like(x) for x in xt]
    import ctypes
    for p, x in zip(plans, xt):
        p.bind_workspace(x.device)
    arr = ctypes.c_void_p * len(plans)
    st = dft3d.lib().dft3d_execute_batched(
        arr(*[p.handle.value for p in plans]), arr(*[x.data_ptr() for x in xt]),
        arr(*[o.data_ptr() for o in outs]), len(plans), -1,
        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    say("bounded wait status", st)
    assert st in (dft3d.OK, dft3d.ERR_HIP)
    for p in plans:
        p.close()
    monkeypatch.delenv("DFT3D_BATCH_SPIN_LIMIT")
    shapes = [(16, 32, 8), (64, 8, 32), (4, 4, 4)]
    xs, xt = make_batch(shapes, 95)
    plans = [dft3d.Plan(s, "pencil", batch_launch=1) for s in shapes]
    outs = [torch.empty_like(x) for x in xt]
    for p, x in zip(plans, xt):
        p.bind_workspace(x.device)
    st = dft3d.lib().dft3d_execute_batched(
        (ctypes.c_void_p * 3)(*[p.handle.value for p in plans]),
        (ctypes.c_void_p * 3)(*[x.data_ptr() for x in xt]),
        (ctypes.c_void_p * 3)(*[o.data_ptr() for o in outs]), 3, -1,
        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == dft3d.OK
    check_against_oracle(xs, outs, -1)
    for p in plans:
        p.close()


@pytest.mark.parametrize("launch", ["levels", "persistent"])
def test_distinct_plans_sharing_one_workspace(launch):
    """Distinct plans bound to one caller workspace are ordered for
    dft3d_execute; in one batched call their passes run together, so the
    library gives all but the first a workspace of their own."""
    shapes = [(16, 32, 64), (32, 16, 64), (64, 32, 16)]
    say("case shared workspace", launch, shapes)
    xs, xt = make_batch(shapes, 130)
    plans = [dft3d.Plan(s, "pencil", batch_launch=1 if launch == "persistent" else 0)
             for s in shapes]
    need = max(p.workspace_size() for p in plans)
    shared = torch.empty(need, dtype=torch.uint8, device="cuda")
    import ctypes
    L = dft3d.lib()
    for p in plans:
        assert L.dft3d_set_workspace(p.handle, shared.data_ptr(), need) == dft3d.OK
    outs = [torch.empty_like(x) for x in xt]
    arr = ctypes.c_void_p * len(plans)
    for sign in (-1, 1):
        st = L.dft3d_execute_batched(
            arr(*[p.handle.value for p in plans]), arr(*[x.data_ptr() for x in xt]),
            arr(*[o.data_ptr() for o in outs]), len(plans), sign,
            torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert st == dft3d.OK
        check_against_oracle(xs, outs, sign)
    for p in plans:
        p.close()


@pytest.mark.parametrize("schedule", ["pencil", "slab", "auto"])
def test_level_batched_mixed_shapes(schedule):
    """One launch per pass level for a batch of mixed shapes: every result
    against the oracle and against its own single-plan execution."""
    shapes = [(32, 64, 128), (128, 32, 64), (64, 64, 64), (8, 16, 4), (2, 2, 2),
              (1, 1, 1), (32, 32, 32), (128, 128, 16)]
    say("case level-batched", schedule, shapes)
    xs, xt = make_batch(shapes, 40)
    ys = dft3d.fftn_batched(xt, schedule=schedule)
    torch.cuda.synchronize()
    check_against_oracle(xs, ys, -1)
    for x, y in zip(xt, ys):
        single = dft3d.fftn(x, schedule=schedule)
        torch.cuda.synchronize()
        assert oracle.rel_l2(y.cpu().numpy(), single.cpu().numpy()) <= oracle.tol(x.numel())


def test_level_batched_96_problems_repeat_and_inverse():
    """The uneven 96-problem workload, called repeatedly with new inputs and
    new output buffers (descriptors refreshed each call), then inverse."""
    shapes = inputs.batch_shapes(96, 104)
    say("case level-batched 96", len(shapes))
    xs, xt = make_batch(shapes, 500)
    outs = [torch.empty_like(x) for x in xt]
    for rep in range(3):
        dft3d.fftn_batched(xt, outs=outs)
        torch.cuda.synchronize()
        for i in range(rep, 96, 7):
            ref = oracle.dft3d(xs[i].astype(np.complex128), -1, "fft")
            assert oracle.rel_l2(outs[i].cpu().numpy(), ref) <= oracle.tol(xs[i].size), (rep, i)
        for i in range(96):
            xs[i] = inputs.uniform_c64(shapes[i], 900 + 96 * rep + i)
            xt[i].copy_(torch.from_numpy(xs[i]))
    outs2 = dft3d.fftn_batched(xt, inverse=True)
    torch.cuda.synchronize()
    for i in range(0, 96, 11):
        ref = oracle.dft3d(xs[i].astype(np.complex128), +1, "fft")
        assert oracle.rel_l2(outs2[i].cpu().numpy(), ref) <= oracle.tol(xs[i].size)


def test_level_batched_every_plane_shape():
    """Slab plans of every plane shape the batched plane kernel covers
    ({32, 64, 128} squared), with a few planes each, in one batch; forward
    and inverse against the oracle."""
    shapes = [(n0, n1, n2) for n1 in (32, 64, 128) for n2 in (32, 64, 128)
              for n0 in (2,)] + [(4, 16, 64), (2, 128, 16)]
    say("case plane shapes", shapes)
    xs, xt = make_batch(shapes, 70)
    for inv, sign in ((False, -1), (True, 1)):
        ys = dft3d.fftn_batched(xt, schedule="slab", inverse=inv)
        torch.cuda.synchronize()
        check_against_oracle(xs, ys, sign)
