"""Optional roctx ranges (HRLB_TRACE): off by default, on when the variable is set and the
roctx library loads; host-side only, no GPU needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = ("import sys; sys.path.insert(0, {root!r}); from paper_1702_01335_amd import hrlb; "
         "q = hrlb.Quadrature(4, 3, 3); print('trace', int(hrlb.trace_status()))")


def _status(env_value):
    env = dict(os.environ)
    env.pop('HRLB_TRACE', None)
    if env_value is not None:
        env['HRLB_TRACE'] = env_value
    r = subprocess.run([sys.executable, '-c', PROBE.format(root=ROOT)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    return int(r.stdout.strip().splitlines()[-1].split()[1])


def _roctx_loadable():
    import ctypes
    try:
        ctypes.CDLL('librocprofiler-sdk-roctx.so.1')
        return True
    except OSError:
        return False


def test_ranges_are_off_without_the_variable():
    assert _status(None) == 0
    assert _status('0') == 0


@pytest.mark.skipif(not _roctx_loadable(), reason='the roctx library is not installed here')
def test_ranges_are_on_with_the_variable():
    assert _status('1') == 1
