"""Host-side logic of bench.py (no GPU): the one-GPU contract and the provenance rule of the
reported HBM traffic (profiled byte counters are used only for the launch shape and the
kernel source they were taken from)."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TAG = 'stage_kernel_couette_shakhov_s256_v800_b256'


def _bench():
    spec = importlib.util.spec_from_file_location('bench_under_test', os.path.join(ROOT, 'bench.py'))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out['n_gpus'] == 2 and 'one GPU' in out['error']


def test_committed_profiles_match_the_kernel_source():
    """Every committed traffic file was taken from the kernel source in the tree, so the
    benchmark reports its bytes; each names its launch shape and its three stage kernels."""
    src = open(os.path.join(ROOT, 'paper_1702_01335_amd', 'csrc', 'kernels.hip'), 'rb').read()
    sha = hashlib.sha256(src).hexdigest()
    files = [f for f in os.listdir(os.path.join(ROOT, 'profiles')) if f.startswith(TAG) and f.endswith('_traffic.json')]
    assert files
    bench = _bench()
    for f in files:
        tr = json.load(open(os.path.join(ROOT, 'profiles', f)))
        assert tr['kernel_source_sha256'] == sha, f
        assert len(tr['stage_kernels']) == 3, f
        assert os.path.exists(os.path.join(ROOT, 'profiles', f.replace('_traffic.json', '.md'))), f
        c, w = tr['launch']['cells'], tr['launch']['waves']
        t = bench.profiled_traffic(TAG, 1.0e9, c, w)
        assert t is not None and t['bytes_per_launch'] > 1.0e9, f
        assert all(b is not None and b > 5.0e8 for b in t['per_stage_bytes']), f
        assert t['source'] == f'profiles/{TAG}_c{c}w{w}.md'


def test_unprofiled_shape_or_changed_source_reports_no_traffic(tmp_path, monkeypatch):
    bench = _bench()
    assert bench.profiled_traffic(TAG, 1.0e9, 3, 3) is None  # shape never profiled
    # a copy of the tree whose kernel source differs from the profiled one
    (tmp_path / 'profiles').mkdir()
    (tmp_path / 'paper_1702_01335_amd' / 'csrc').mkdir(parents=True)
    name = f'{TAG}_c64w1_traffic.json'
    (tmp_path / 'profiles' / name).write_text(open(os.path.join(ROOT, 'profiles', name)).read())
    (tmp_path / 'paper_1702_01335_amd' / 'csrc' / 'kernels.hip').write_text('// another kernel source\n')
    monkeypatch.setattr(bench, 'ROOT', str(tmp_path))
    assert bench.profiled_traffic(TAG, 1.0e9, 64, 1) is None
