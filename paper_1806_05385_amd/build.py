"""Build libpr.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, 'csrc', 'pr_api.hip')
LIB = os.path.join(HERE, 'libpr.so')

FLAGS = [
    '-O3', '-std=c++17', '-fPIC', '-shared', '--offload-arch=gfx950',
    # keep packed-FP32 VALU instructions out of the generated code
    '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
    # matrix products read and write VGPRs directly (no AGPR copies)
    '-mllvm', '-amdgpu-mfma-vgpr-form',
    '-Wno-unused-command-line-argument',
]


def build(verbose: bool = False) -> str:
    tmp = LIB + '.tmp'
    cmd = ['hipcc', *FLAGS, '-I', os.path.join(ROOT, 'include'), '-I', os.path.join(HERE, 'csrc'),
           '-o', tmp, SRC]
    if verbose:
        print(' '.join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    build(verbose=True)
    sys.exit(0)
