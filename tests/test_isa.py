"""Static checks of the gfx950 code the library's kernels compile to (device
assembly from hipcc -S, no GPU needed).

* No flat memory instructions in any kernel: every buffer is global memory, and
  a pointer whose address space the compiler cannot see (one read from memory,
  or passed through inline asm) turns its loads into flat loads, which halved
  the throughput of the entry kernels once.
* No register spills and no scratch arrays in the kernels on the hot paths
  (entry generation for the HSS levels, the matrix-free product, the CPQR
  step and the whole-box CPQR, the batched products, the Gauss-Jordan
  inverses and the panel steps of the dense root).
  The shape-derivative pair kernel is the exception on purpose: at three waves
  per SIMD it spills 23 VGPRs and runs in 2.20 ms on the N = 8192 gradient
  workload, against 2.46 ms at two waves per SIMD without spills."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_00790_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SOURCES = ["assemble.hip", "hss_kernels.hip", "gen_api.hip", "adjoint.hip"]
NO_SPILL = ["k_matvec_partial", "k_gen_jobs", "k_cpqr_step_reg", "k_cpqr_fused", "k_gemm", "k_gemv",
            "k_gauss_jordan", "k_sketch", "k_interp", "k_shape_nodes"]


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = {}
    d = tmp_path_factory.mktemp("isa")
    for src in SOURCES:
        s = os.path.join(d, src + ".s")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O3", f"-I{os.path.join(ROOT, 'include')}",
                        f"-I{CSRC}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "--cuda-device-only", "-S", "-o", s, os.path.join(CSRC, src)],
                       check=True, capture_output=True)
        out[src] = open(s).read()
    return out


def kernels(text):
    """(name, body, metadata) of every kernel in one assembly file."""
    res = []
    for m in re.finditer(r"^(_Z\S+):", text, re.M):
        name = m.group(1)
        end = text.find(".Lfunc_end", m.end())
        meta = re.search(r"\.name:\s+" + re.escape(name) + r"\n(.*?)(?=\n\s+- \.|\n\.end_amdgpu_metadata)",
                         text, re.S)
        res.append((name, text[m.end():end], meta.group(1) if meta else ""))
    return res


def test_no_flat_memory_instructions(asm):
    for src, text in asm.items():
        ks = kernels(text)
        assert ks, src
        for name, body, _ in ks:
            flat = re.findall(r"^\s*(flat_\w+)", body, re.M)
            assert not flat, f"{src}: {name} uses {sorted(set(flat))}"


def test_hot_kernels_do_not_spill(asm):
    seen = set()
    for src, text in asm.items():
        for name, _, meta in kernels(text):
            hit = [k for k in NO_SPILL if k in name]
            if not hit:
                continue
            seen.update(hit)
            spill = re.search(r"\.vgpr_spill_count:\s+(\d+)", meta)
            assert spill is not None, name
            assert int(spill.group(1)) == 0, f"{name} spills {spill.group(1)} VGPRs"
            # no private (scratch) arrays either: a register array indexed at run
            # time lands there, which once made the Gauss-Jordan kernel 3x slower
            priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", meta)
            assert priv is not None and int(priv.group(1)) == 0, f"{name} uses {priv.group(1)} B of scratch"
    assert seen == set(NO_SPILL)
