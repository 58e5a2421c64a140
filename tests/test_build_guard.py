"""The fused substage kernel is built without scratch memory (the build
checks the device assembly); the check itself finds scratch accesses where
they exist."""
import os

import pytest

from paper_1908_08557_amd import build as B


def test_substage_kernels_use_no_scratch():
    counts = B.scratch_report(os.path.join(B.CSRC, "substage.hip"), "k_substage")
    assert len(counts) >= 18          # every precision / boundary / stage variant
    assert all(n == 0 for n in counts.values()), counts


def test_scratch_report_sees_spills(tmp_path):
    # a kernel that indexes a private array dynamically must use scratch
    src = tmp_path / "spill.hip"
    src.write_text(
        "#include <hip/hip_runtime.h>\n"
        "__global__ void k_spill_probe(double* o, int i) {\n"
        "  double a[64];\n"
        "  for (int j = 0; j < 64; ++j) a[j] = o[j * threadIdx.x];\n"
        "  o[threadIdx.x] = a[(i + threadIdx.x) & 63];\n"
        "}\n")
    counts = B.scratch_report(str(src), "k_spill_probe")
    assert counts and all(n > 0 for n in counts.values())
