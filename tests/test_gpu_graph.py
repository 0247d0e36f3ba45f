"""HIP graph capture of dft3d_execute: a plan whose workspace is bound and
which has run once only launches kernels, so torch's graph capture (a HIP
graph on ROCm) records the passes, and every replay must reproduce the
eager result bit for bit (same kernels, same inputs), also with eager work
on the same plan between replays and with new input values."""
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
    assert "libdft3d.so" in open("/proc/self/maps").read()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape,schedule,layout", [
    ((64, 64, 64), "pencil", "natural"),
    ((32, 64, 128), "slab", "natural"),
    ((64, 32, 16), "volumetric", "shuffled"),
    ((512, 512, 512), "auto", "natural"),   # persistent streaming kernels
    ((100, 30, 17), "pencil", "natural"),   # mixed-radix and Bluestein passes
    ((1000, 96, 12), "auto", "natural"),    # mixed radix with radices 10 and 16
])
def test_graph_replay_matches_eager(shape, schedule, layout):
    say("case graph", shape, schedule, layout)
    x = torch.from_numpy(inputs.uniform_c64(shape, 41)).cuda()
    p = dft3d.Plan(shape, schedule, layout=layout)
    p.bind_workspace(x.device)
    for inverse in (False, True):
        eager = torch.empty_like(x)
        p.execute(x, eager, inverse=inverse)      # first run outside capture
        torch.cuda.synchronize()
        y = torch.empty_like(x)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                p.execute(x, y, inverse=inverse)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(3):
            y.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, eager), (rep, inverse)
            other = torch.empty_like(x)           # eager work between replays
            p.execute(eager, other, inverse=not inverse)
            torch.cuda.synchronize()
        # new values in the captured input buffer: the replay transforms them
        x2 = inputs.uniform_c64(shape, 42)
        x.copy_(torch.from_numpy(x2))
        g.replay()
        torch.cuda.synchronize()
        if x.numel() <= (1 << 21):
            sign = 1 if inverse else -1
            pow2 = all(n & (n - 1) == 0 for n in shape)
            # other lengths: direct sums, and twice the bar (a Bluestein axis
            # carries about twice the rounding levels of its length)
            ref = oracle.dft3d(x2.astype(np.complex128), sign, "fft" if pow2 else "direct")
            got = y.cpu().numpy()
            if layout == "shuffled":
                f = dft3d.shuffle_factors(shape)
                ref = oracle.to_shuffled(ref, f) if not inverse else oracle.dft3d(
                    oracle.from_shuffled(x2.astype(np.complex128), f), +1, "fft")
            assert oracle.rel_l2(got, ref) <= oracle.tol(x.numel()) * (1 if pow2 else 2)
        else:
            eager2 = torch.empty_like(x)
            p.execute(x, eager2, inverse=inverse)
            torch.cuda.synchronize()
            assert torch.equal(y, eager2)
        x.copy_(torch.from_numpy(inputs.uniform_c64(shape, 41)))
        del g
    p.close()


@pytest.mark.parametrize("launch", ["levels", "persistent"])
def test_batched_graph_replay_matches_eager(launch):
    """Batched execution captured after an eager call with the same buffers:
    replays reproduce the eager result bit for bit, also after eager batched
    calls with other output buffers in between (which must not disturb the
    captured descriptors), and transform new values put in the inputs."""
    shapes = [(32, 64, 128), (64, 64, 64), (8, 16, 4), (128, 32, 16), (32, 32, 32)]
    print("case batched graph", launch, shapes, flush=True)
    xs = [torch.from_numpy(inputs.uniform_c64(s, 50 + i)).cuda() for i, s in enumerate(shapes)]
    outs = [torch.empty_like(x) for x in xs]
    for inverse in (False, True):
        dft3d.fftn_batched(xs, outs=outs, inverse=inverse, launch=launch)     # eager: descriptors on device
        torch.cuda.synchronize()
        eager = [o.clone() for o in outs]
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                dft3d.fftn_batched(xs, outs=outs, inverse=inverse, launch=launch)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                assert torch.equal(o, e), rep
            other = dft3d.fftn_batched(xs, inverse=inverse, launch=launch)   # other output buffers
            torch.cuda.synchronize()
            for o, e in zip(other, eager):
                assert torch.equal(o, e)
        new = [inputs.uniform_c64(sh, 80 + i) for i, sh in enumerate(shapes)]
        for x, n in zip(xs, new):
            x.copy_(torch.from_numpy(n))
        g.replay()
        torch.cuda.synchronize()
        sign = 1 if inverse else -1
        for o, n in zip(outs, new):
            ref = oracle.dft3d(n.astype(np.complex128), sign, "fft")
            assert oracle.rel_l2(o.cpu().numpy(), ref) <= oracle.tol(n.size)
        for i, sh in enumerate(shapes):
            xs[i].copy_(torch.from_numpy(inputs.uniform_c64(sh, 50 + i)))
        del g


def test_batched_capture_without_prior_call_is_refused():
    shapes = [(16, 16, 16), (8, 8, 8)]
    xs = [torch.zeros(s, dtype=torch.complex64, device="cuda") for s in shapes]
    outs = [torch.empty_like(x) for x in xs]
    plans = [dft3d.Plan(s, "pencil") for s in shapes]     # fresh plans: nothing on device
    for p, x in zip(plans, xs):
        p.bind_workspace(x.device)
    import ctypes
    arr = ctypes.c_void_p * len(plans)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    st = None
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            st = dft3d.lib().dft3d_execute_batched(
                arr(*[p.handle.value for p in plans]), arr(*[x.data_ptr() for x in xs]),
                arr(*[o.data_ptr() for o in outs]), len(plans), -1, s.cuda_stream)
    assert st == dft3d.ERR_UNSUPPORTED_SCHEDULE
    for p in plans:
        p.close()
