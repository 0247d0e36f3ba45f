"""Error paths on the GPU, forced from the host (no kernel is made to
fail): DFT3D_FAULT_INJECT=alloc|upload|launch makes that step of the
library fail, DFT3D_MAX_WORKSPACE_BYTES caps plan-owned workspaces.  Every
failing call returns its status, leaves the output handle NULL, and leaks no
device memory (the device's free memory, which counts the library's own
allocations, is unchanged after many failing calls)."""
import ctypes

import pytest

from paper_1904_10119_amd import dft3d

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def make_plan(shape, schedule=2):
    h = ctypes.c_void_p()
    st = dft3d.lib().dft3d_plan(*shape, schedule, 0, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("step,status", [("alloc", dft3d.ERR_OUT_OF_MEMORY),
                                         ("upload", dft3d.ERR_HIP)])
def test_plan_failures_leak_nothing(monkeypatch, step, status):
    print("case fault", step, flush=True)
    shape = (256, 256, 256)
    st, h = make_plan(shape)          # warm the runtime and the module first
    assert st == dft3d.OK
    dft3d.lib().dft3d_destroy(h)
    before = free_bytes()
    monkeypatch.setenv("DFT3D_FAULT_INJECT", step)
    for _ in range(200):
        st, h = make_plan(shape)
        assert st == status
        assert h.value is None
    monkeypatch.delenv("DFT3D_FAULT_INJECT")
    assert free_bytes() >= before - (2 << 20)
    st, h = make_plan(shape)          # the library still works
    assert st == dft3d.OK
    dft3d.lib().dft3d_destroy(h)


def test_option_change_failure_keeps_plan(monkeypatch):
    """A failing rebuild (table upload) leaves the previous pass list in
    force and usable."""
    st, h = make_plan((64, 64, 64))
    assert st == dft3d.OK
    L = dft3d.lib()
    monkeypatch.setenv("DFT3D_FAULT_INJECT", "upload")
    assert L.dft3d_plan_set_option(h, dft3d.OPT_PRECISION, 3) == dft3d.ERR_HIP
    monkeypatch.delenv("DFT3D_FAULT_INJECT")
    v = ctypes.c_int64()
    assert L.dft3d_plan_get_option(h, dft3d.OPT_PRECISION, ctypes.byref(v)) == dft3d.OK
    assert v.value == 0
    x = torch.ones((64, 64, 64), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    st = L.dft3d_execute(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), -1,
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == dft3d.OK
    assert abs(complex(y[0, 0, 0].item()) - 64 ** 3) < 1e-3 * 64 ** 3
    L.dft3d_destroy(h)


@pytest.mark.parametrize("step,env,status", [
    ("workspace alloc", ("DFT3D_FAULT_INJECT", "alloc"), dft3d.ERR_OUT_OF_MEMORY),
    ("workspace cap", ("DFT3D_MAX_WORKSPACE_BYTES", str(1 << 20)), dft3d.ERR_OUT_OF_MEMORY),
    ("launch", ("DFT3D_FAULT_INJECT", "launch"), dft3d.ERR_HIP)])
def test_execute_failures_leak_nothing(monkeypatch, step, env, status):
    print("case execute fault", step, flush=True)
    shape = (128, 128, 128)            # 16 MiB of workspace on the pencil schedule
    L = dft3d.lib()
    x = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    before = free_bytes()
    for _ in range(50):
        st, h = make_plan(shape)       # the plan itself is made without the fault
        assert st == dft3d.OK
        monkeypatch.setenv(*env)
        st = L.dft3d_execute(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                             -1, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        monkeypatch.delenv(env[0])
        assert st == status
        assert L.dft3d_destroy(h) == dft3d.OK
    assert free_bytes() >= before - (2 << 20)


def test_workspace_cap_allows_small_plans(monkeypatch):
    """Below the cap the plan allocates and runs as usual; slab plans need
    no workspace and ignore the cap."""
    monkeypatch.setenv("DFT3D_MAX_WORKSPACE_BYTES", str(64 << 20))
    x = torch.ones((64, 64, 64), dtype=torch.complex64, device="cuda")
    for sch in ("pencil", "slab"):
        p = dft3d.Plan((64, 64, 64), sch)
        y = torch.empty_like(x)
        p._ws = None
        L = dft3d.lib()
        st = L.dft3d_execute(p.handle, ctypes.c_void_p(x.data_ptr()),
                             ctypes.c_void_p(y.data_ptr()), -1,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert st == dft3d.OK
        p.close()
