"""Source-level checks of the HIP kernels that need no GPU."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS = os.path.join(ROOT, "paper_1910_01997_amd", "csrc", "sgn_kernels.hip")


def _norm(text):
    lines = []
    for line in text.splitlines():
        line = re.sub(r"//.*", "", line).strip()
        if line:
            lines.append(line)
    return lines


def test_gn_kernel_owner_step_copy_equals_the_function():
    """gn_kernel writes the owner-lane step out by hand (register
    allocation); it must stay the same code as owner_step, which the disc
    kernel calls."""
    src = open(KERNELS).read()
    a = src.index("__device__ __forceinline__ bool owner_step(")
    body = src[src.index("{", a) + 1:src.index("\n}\n", a)]
    fn = _norm(body)
    assert fn[0] == "bool cand = false;" and fn[-1] == "return cand;"
    fn = fn[1:-1]
    b = src.index("// owner_step body begin")
    e = src.index("// owner_step body end")
    copy = _norm(src[b:e])
    assert copy[0] == "const float* sm = lsm + own * SM_WORDS;"
    assert copy[1:] == fn
