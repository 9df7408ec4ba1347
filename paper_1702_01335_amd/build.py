"""Build libhrlb.so in-tree for gfx950 (MI355X).

    python -m paper_1702_01335_amd.build

Host C++ (quadrature tables, C ABI) is compiled by g++ against the HIP headers, the
kernels (solver and warm-start network, with its C ABI) by hipcc for gfx950 with
packed-FP32 instruction selection disabled, and the objects are linked by hipcc into
paper_1702_01335_amd/libhrlb.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(HERE, '_build')
LIB = os.path.join(HERE, 'libhrlb.so')
ROCM = os.environ.get('ROCM_PATH', '/opt/rocm')
HIPCC = os.path.join(ROCM, 'bin', 'hipcc')

INC = ['-I', os.path.join(ROOT, 'include'), '-I', CSRC]
HIP_DEVICE_FLAGS = ['--offload-arch=gfx950', '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']


def _run(cmd, verbose):
    if verbose:
        print(' '.join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in ('quadrature.cpp', 'capi.cpp'):
        obj = os.path.join(BUILD, src.replace('.cpp', '.o'))
        _run(['g++', '-O2', '-std=c++17', '-fPIC', '-Wall', '-D__HIP_PLATFORM_AMD__', '-I', os.path.join(ROCM, 'include')]
             + INC + ['-c', os.path.join(CSRC, src), '-o', obj], verbose)
        objs.append(obj)
    for src in ('kernels.hip', 'mlp.hip'):
        kobj = os.path.join(BUILD, src.replace('.hip', '.o'))
        _run([HIPCC, '-O3', '-std=c++17', '-fPIC'] + HIP_DEVICE_FLAGS + INC + ['-c', os.path.join(CSRC, src), '-o', kobj],
             verbose)
        objs.append(kobj)
    tmp = LIB + '.tmp'
    _run([HIPCC, '-shared', '-fPIC', '--offload-arch=gfx950'] + objs + ['-o', tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    build(verbose='-q' not in sys.argv)
