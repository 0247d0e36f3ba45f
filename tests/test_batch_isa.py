"""CPU check of the compiled control flow of the one-launch batched kernel.

The kernel's ticket loop must keep every branch around its barriers
wave-uniform.  An earlier form did its per-workgroup work in
`if (threadIdx.x == 0)` blocks at the start and at the end of the loop; the
compiler merged the two across the back-edge and turned the rest of the loop
into an inner loop around the barriers that runs with lane 0 of the first
wave masked off (an `s_andn2_b64 exec, exec, ...` loop exit ahead of the
barriers).  That inner loop re-ran the same tile forever: the launch never
finished.  This test compiles the kernel (device code only, gfx950) and
checks that no such divergent loop exit comes before the last barrier."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_10119_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def kernel_asm(tmp_path, name):
    out = tmp_path / "batch.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "--offload-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-S", os.path.join(CSRC, "batch.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=CSRC)
    assert r.returncode == 0, r.stderr[-2000:]
    text = out.read_text()
    m = re.search(r"^(_ZN5dft3d\d+%s\w*):.*?$(.*?)s_endpgm" % name, text, re.S | re.M)
    assert m, name
    return m.group(2).splitlines()


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_persistent_batched_loop_has_no_divergent_exit_before_barriers(tmp_path):
    lines = kernel_asm(tmp_path, "batch_persistent_kernel")
    barriers = [i for i, l in enumerate(lines) if l.strip() == "s_barrier"]
    assert len(barriers) >= 2, "expected the two barriers of the ticket loop"
    last = barriers[-1]
    masked_exits = [i for i, l in enumerate(lines[:last])
                    if re.match(r"\s*s_andn2_b64 exec, exec, ", l)]
    assert not masked_exits, [lines[i] for i in masked_exits]
