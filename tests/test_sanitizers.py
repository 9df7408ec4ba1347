"""The host code of the C ABI (argument checks, quadrature construction, carve-up sizes)
built with AddressSanitizer and UndefinedBehaviorSanitizer by g++ and run without a GPU
(tests/sanitize/host_abi.cpp).  The kernels' object file comes from the normal build; only
the host sources are instrumented."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, 'paper_1702_01335_amd')
ROCM = os.environ.get('ROCM_PATH', '/opt/rocm')


@pytest.mark.skipif(shutil.which('g++') is None, reason='needs g++')
def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    kobj = os.path.join(PKG, '_build', 'kernels.o')
    if not os.path.exists(kobj):
        pytest.skip('library not built (python -m paper_1702_01335_amd.build)')
    exe = str(tmp_path / 'host_abi')
    cmd = ['g++', '-O1', '-g', '-std=c++17', '-fsanitize=address,undefined', '-fno-sanitize-recover=undefined',
           '-fno-omit-frame-pointer', '-D__HIP_PLATFORM_AMD__', '-I', os.path.join(ROCM, 'include'),
           '-I', os.path.join(ROOT, 'include'), '-I', os.path.join(PKG, 'csrc'),
           os.path.join(ROOT, 'tests', 'sanitize', 'host_abi.cpp'), os.path.join(PKG, 'csrc', 'capi.cpp'),
           os.path.join(PKG, 'csrc', 'quadrature.cpp'), kobj, '-L', os.path.join(ROCM, 'lib'), '-lamdhip64',
           '-Wl,-rpath,' + os.path.join(ROCM, 'lib'), '-o', exe]
    subprocess.run(cmd, check=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS='detect_leaks=0:abort_on_error=0', UBSAN_OPTIONS='print_stacktrace=1')
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == 'ok'
    assert 'runtime error' not in r.stderr and 'AddressSanitizer' not in r.stderr
