"""Benchmark of the RK3 time step of the half-range LB Couette solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--workload NAME]

A step is one TVD RK3 step (three stages, each a closure launch and a stage launch) of
every instance of the batch; the batch is B independent seeded instances of one
workload, resident in HBM before timing starts.  Prints one JSON line with the
throughput in G (node x velocity) pair-updates per second, the roofline record of the
dominant kernel (the stage kernel, timed with HIP events on the stream it runs on) and
the oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

# the oracle baseline runs single-threaded; fix the BLAS pool before numpy loads
os.environ.setdefault('OPENBLAS_NUM_THREADS', '1')
os.environ.setdefault('OMP_NUM_THREADS_ORACLE', '1')

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
BYTES_PER_PAIR_STEP = 64   # algorithmic: stage 1 16 B, stages 2-3 24 B each (read F_in, F_l; write F_out)
STAGE_BYTES = (16, 24, 24)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=100)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--batch', type=int, default=256)
    ap.add_argument('--workload', default='couette_shakhov_s256_v800')
    ap.add_argument('--cells', type=int, default=0)
    ap.add_argument('--waves', type=int, default=0)
    ap.add_argument('--scheme', default=None, choices=('weno5', 'linear5', 'upwind2'),
                    help="x advection scheme instead of the workload's (to time what the scheme costs; the "
                         "profiled byte counts then do not apply)")
    ap.add_argument('--no-cpu', action='store_true')
    ap.add_argument('--eager', action='store_true', help='launch kernels one by one instead of replaying a HIP graph')
    ap.add_argument('--no-tune', action='store_true', help='keep the default launch shape instead of autotuning it')
    ap.add_argument('--tune-cache', default=None,
                    help='JSON-lines cache of autotuned launch shapes; a shape found there is used without timing '
                         '(default: time every shape on this GPU)')
    ap.add_argument('--copy-probe-mib', type=int, default=0,
                    help='also run one device copy of this size (calibrates HBM byte counters under a profiler)')
    ap.add_argument('--cpu-seconds', type=float, default=12.0,
                    help='seconds of oracle stepping for each of the one-core and all-core CPU figures')
    ap.add_argument('--cpu-cores', type=int, default=0,
                    help='processes of the all-core CPU figure (default: the cores this process may use, at most 16)')
    ap.add_argument('--cpu-suite', action='store_true',
                    help='only time the oracle on the host on the measurement plan\'s cases (long; no GPU use)')
    ap.add_argument('--no-sweep', action='store_true', help='skip the ragged-sweep measurements')
    ap.add_argument('--sweep-instances', type=int, default=256)
    ap.add_argument('--steady-instances', type=int, default=16)
    ap.add_argument('--no-warm', action='store_true', help='skip the learned warm-start measurement')
    ap.add_argument('--no-workloads', action='store_true', help='skip the per-workload table')
    ap.add_argument('--warm-train', type=int, default=2000, help='instances whose steady states train the network')
    ap.add_argument('--warm-heldout', type=int, default=200)
    ap.add_argument('--warm-steps', type=int, default=10000, help='AdamW steps of the network')
    return ap.parse_args()


def make_solver(wl, batch, device):
    import numpy as np
    import torch
    from paper_1702_01335_amd import hrlb, inputs
    q = hrlb.ReducedQuadrature(wl['Qx'], wl['Qy']) if wl.get('reduced') else hrlb.Quadrature(wl['Qx'], wl['Qy'], wl['Qz'])
    S = wl['S']
    r = torch.empty((batch, S, q.V), dtype=torch.float64, device=device)
    for b in range(batch):
        r[b] = torch.from_numpy(inputs.perturbation(1000 + b, (S, q.V)))
    params = [hrlb.make_params(**wl['params']) for _ in range(batch)]
    solver = hrlb.Solver(q, S, wl['scheme'], params, device=device, perturb=r, eps=0.05)
    del r
    return q, solver


def time_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    solver.synchronize()
    torch.cuda.synchronize()
    s = solver.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    solver.step(steps)
    e1.record(s)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def profiled_traffic(tag, bytes_per_launch, cells, waves):
    """HBM bytes per stage-kernel launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes of this launch shape (profiles/<tag>_c<cells>w<waves>_traffic.json), or None when
    that shape was not profiled or the kernel source differs from the one profiled."""
    import hashlib
    path = os.path.join(ROOT, 'profiles', f'{tag}_c{cells}w{waves}_traffic.json')
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    src = open(os.path.join(ROOT, 'paper_1702_01335_amd', 'csrc', 'kernels.hip'), 'rb').read()
    if hashlib.sha256(src).hexdigest() != tr['kernel_source_sha256']:
        return None
    if tr.get('launch') != {'cells': cells, 'waves': waves}:
        return None
    ks = tr['stage_kernels'].values()
    t = sum(k['fetch_bytes'] + k['write_bytes'] for k in ks) / len(ks)
    # counted bytes of each RK3 stage: the stage is the second template argument of the name
    per_stage = [None, None, None]
    for name, k in tr['stage_kernels'].items():
        st = int(name.split('<')[1].split(',')[1])
        per_stage[st - 1] = k['fetch_bytes'] + k['write_bytes']
    return {'bytes_per_launch': t, 'over_algorithmic': t / bytes_per_launch, 'per_stage_bytes': per_stage,
            'source': f'profiles/{tag}_c{cells}w{waves}.md'}


def delivered_bandwidth(device, mib=512, reps=10):
    """What this GPU's HBM delivers to plain streams, timed now: a device copy (one read, one
    write stream, like the first RK3 stage) and an add (two reads, one write, like stages 2
    and 3) of mib-MiB float64 arrays, in bytes/s."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device=device)
    y = torch.ones_like(x)
    z = torch.empty_like(x)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    copy = 2 * n * 8 / timed(lambda: z.copy_(x))
    add = 3 * n * 8 / timed(lambda: torch.add(x, y, out=z))
    del x, y, z
    torch.cuda.empty_cache()
    return copy, add


def sweep_section(n_inst, n_steady, steps):
    """Ragged sweep measurements.  Throughput: n_inst instances drawn from the sweep
    distribution (kn log-uniform in [0.01, 100], u_w in [0.05, 0.6], omega in
    {0.5, 0.72, 0.81, 1}, Qx in {4, 8, 16, 32}, S in {64, 128, 256}, Qy = Qz = 5, upwind2)
    advanced as one autotuned batch, against the same groups stepped one after
    another and against every instance stepped alone.  Time to steady state: n_steady
    instances of the same distribution restricted to S = 64 and Qx in {4, 8}, run to
    residual 1e-10 as one batch that retires converged instances, against the same
    instances run one at a time."""
    import numpy as np
    import torch
    from paper_1702_01335_amd import hrlb
    from paper_1702_01335_amd.sweep import Sweep, sample
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        fn(2)
        torch.cuda.synchronize()
        e0.record()
        fn(k)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / k

    # the same instances with the survey's reading of the sweep's scheme and grid (WENO-5 on
    # the A = 0.98 tanh grid): throughput only (the epsilon-free WENO-5 residual need not
    # fall to 1e-10, so the time to steady state is measured with upwind-2 below)
    sw = Sweep(sample(n_inst, 20170204), scheme='weno5', A=0.98)
    cw, ww, _ = sw.autotune(probe_steps=5)
    ms_w = timed(sw.batch.step, steps)
    weno = dict(scheme='weno5', A=0.98, launch=dict(cells=cw, waves=ww, graph=True), batched_ms_per_step=ms_w,
                value=sw.pairs() / ms_w / 1e6, unit='G pair-updates/s')
    del sw
    torch.cuda.empty_cache()
    sw = Sweep(sample(n_inst, 20170204))
    cells, waves, _ = sw.autotune(probe_steps=5)
    pairs = sw.pairs()
    ms_b = timed(sw.batch.step, steps)
    ms_g = 0.0
    for _, _, s in sw.groups:
        s.autotune(probe_steps=3)
        s.set_graph(True)
        ms_g += timed(s.step, max(5, steps // 4))
    del sw
    torch.cuda.empty_cache()
    ms_i = 0.0
    sw1 = Sweep(sample(n_inst, 20170204), cells=4)
    for i in sw1.order:
        d = sw1.instances[i]
        s = sw1._solver((d['Qx'], d['S']), [i])
        s.set_graph(True)
        ms_i += timed(s.step, 5)
        del s
    del sw1
    torch.cuda.empty_cache()
    out = dict(instances=n_inst, pairs=pairs, launch=dict(cells=cells, waves=waves, graph=True),
               batched_ms_per_step=ms_b, value=pairs / ms_b / 1e6, unit='G pair-updates/s',
               groups_one_by_one_ms_per_step=ms_g, instances_one_by_one_ms_per_step=ms_i,
               speedup_vs_groups=ms_g / ms_b, speedup_vs_instances=ms_i / ms_b, weno5_stretched=weno)
    if n_steady:
        tol, budget, every = 1e-10, 400000, 1000
        inst = sample(n_steady, 20170206, qx=(4, 8), nodes=(64,))
        sw = Sweep(inst)
        c, w, _ = sw.autotune(probe_steps=5)
        st_b, R_b, wall_b = sw.run_to_steady(tol, budget, every)
        st_p, R_p, wall_p = sw.run_plain(tol, budget, every)
        out['steady'] = dict(instances=n_steady, tol=tol, check_every=every,
                             subset='kn log-uniform [0.01, 100], u_w [0.05, 0.6], omega sampled, Qx in {4, 8}, S = 64',
                             launch=dict(cells=c, waves=w),
                             batched_wall_s=wall_b, plain_wall_s=wall_p, speedup=wall_p / wall_b,
                             converged_batched=int((st_b > 0).sum()), converged_plain=int((st_p > 0).sum()),
                             steps_max=int(st_b.max()), steps_median=float(np.median(st_b)),
                             steps_equal=bool(np.array_equal(st_b, st_p)),
                             max_residual=float(max(R_b.max(), R_p.max())))
    return out


def workloads_section(steps, warmup):
    """Every workload at its own size: one instance (latency-bound: 0.3 to 118 MB per step)
    and a batch large enough to live in HBM rather than in the 256 MB last-level cache.
    Launch shapes autotuned, HIP graph on."""
    import torch
    from paper_1702_01335_amd.workloads import workload
    out = []
    for name, batch in (('couette_bgk_s64_v128', 1), ('couette_bgk_s64_v128', 4096),
                        ('couette_shakhov_s256_v800', 1), ('couette_shakhov_s256_v800', 512),
                        ('couette_shakhov_s512_v3600', 1), ('couette_shakhov_s512_v3600', 64),
                        ('paper_maxwell_s16_v686', 1), ('paper_maxwell_s16_v686', 4096),
                        ('couette_shakhov_s256_reduced', 1), ('couette_shakhov_s256_reduced', 1024),
                        ('paper_sutherland_s16_reduced', 1), ('paper_sutherland_s16_reduced', 8192)):
        wl = workload(name)
        q, s = make_solver(wl, batch, 'cuda:0')
        c, w, _ = s.autotune(probe_steps=3)
        s.set_graph(True)
        ms, _ = time_steps(s, steps, warmup)
        pairs = batch * wl['S'] * q.V
        out.append(dict(workload=name, batch=batch, pairs=pairs, populations_per_node=q.V,
                        velocities_per_node=q.V // 2 if wl.get('reduced') else q.V,
                        launch=dict(cells=c, waves=w), ms_per_step=ms,
                        value=pairs / (ms * 1e-3) / 1e9,
                        hbm_frac_step=pairs * BYTES_PER_PAIR_STEP / (ms * 1e-3) / HBM_PEAK))
        del s
        torch.cuda.empty_cache()
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def warm_section(n_train, n_heldout, train_steps):
    """Learned warm start: n_train instances of the sweep distribution (one velocity set and
    grid: Qx = 8, Qy = Qz = 5, S = 64, upwind2) run to residual 1e-10 as one batch give the
    training rows; the network is trained on the GPU by the library's kernels; n_heldout
    instances of another seed are run to 1e-10 from the equilibrium start and from the
    warm start."""
    import numpy as np
    from paper_1702_01335_amd import warmstart as ws
    X, Y, info = ws.collect(n_train, 20170205)
    progress(f"warm start: collected {info['rows']} rows in {info['wall_s']:.1f} s")
    net, log, t_train = ws.train(X, Y, steps=train_steps)
    flop = 3 * 2 * 4096 * (5 * 256 + 2 * 256 * 256 + 256 * 8) * train_steps
    progress(f"warm start: trained {train_steps} steps in {t_train:.1f} s, loss {log[-1][1]:.2e}")
    res = ws.compare(net, n_heldout, 20170206)
    st_p, st_w = np.array(res.pop('steps_plain')), np.array(res.pop('steps_warm'))
    return dict(collect=info, train=dict(steps=train_steps, batch=4096, wall_s=t_train, loss_first=log[0][1],
                                         loss_last=log[-1][1], tflops=flop / t_train / 1e12,
                                         frac_bf16_peak=flop / t_train / 2.5e15),
                heldout=res)


def _oracle_worker(args):
    """Step one seeded instance of the workload with the oracle for about `seconds`;
    returns (steps, elapsed).  Runs in its own process, single-threaded."""
    wl, seed, seconds = args
    from oracle import solver as sv
    from paper_1702_01335_amd import inputs
    p = sv.Params(Qx=wl['Qx'], Qy=wl['Qy'], Qz=wl['Qz'], S=wl['S'], scheme=wl['scheme'], **wl['params'])
    m = sv.Model(p)
    F = sv.seeded_state(m, inputs.perturbation(seed, (p.S, m.V)), 0.05)
    F = sv.rk3_step(F, m)  # warm-up
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds or n < 2:
        F = sv.rk3_step(F, m)
        n += 1
    return n, time.perf_counter() - t0


def _oracle_job(job):
    """One timing job of the CPU suite, in its own single-threaded process: ('steady', wl,
    budget) runs the workload from the equilibrium start until the residual of a step falls
    below 1e-10 (checked every 1000 steps) or the budget is spent; ('steps', wl, n, seed)
    runs n steps from the seeded start."""
    from oracle import solver as sv
    from paper_1702_01335_amd import inputs
    kind, wl = job[0], job[1]
    p = sv.Params(Qx=wl['Qx'], Qy=wl['Qy'], Qz=wl['Qz'], S=wl['S'], scheme=wl['scheme'], **wl['params'])
    m = sv.Model(p)
    t0 = time.perf_counter()
    if kind == 'steady':
        F, steps, R = sv.run_to_steady(sv.equilibrium_state(m), m, 1e-10, job[2], check_every=1000)
    else:
        F = sv.seeded_state(m, inputs.perturbation(job[3], (p.S, m.V)), 0.05)
        for _ in range(job[2]):
            F = sv.rk3_step(F, m)
        steps, R = job[2], float('nan')
    wall = time.perf_counter() - t0
    return dict(name=wl.get('name', ''), kind=kind, S=p.S, V=m.V, steps=int(steps), residual=float(R), wall_s=wall,
                value=p.S * m.V * steps / wall / 1e9)


def cpu_suite(cores):
    """The oracle's timings of the measurement plan, host only (no GPU): the first workload and
    the paper-shape workload from the equilibrium start to residual 1e-10, the third workload
    for 100 steps, and the 16 sweep instances of the time-to-steady comparison (seed
    20170206, S = 64, Qx in {4, 8}, upwind-2, Courant 0.5) to 1e-10; the jobs run as
    independent single-threaded processes on `cores` cores."""
    import multiprocessing as mp_
    import numpy as np
    from oracle import quadrature as oq
    from paper_1702_01335_amd.sweep import sample
    from paper_1702_01335_amd.workloads import workload
    jobs = []
    for name, budget in (('couette_bgk_s64_v128', 400000), ('paper_maxwell_s16_v686', 200000)):
        wl = dict(workload(name), name=name)
        jobs.append(('steady', wl, budget))
    jobs.append(('steps', dict(workload('couette_shakhov_s512_v3600'), name='couette_shakhov_s512_v3600'), 100, 3))
    for k, d in enumerate(sample(16, 20170206, qx=(4, 8), nodes=(64,))):
        dt = 0.5 * (1.0 / (2 * d['S'])) / float(np.abs(oq.x_axis(d['Qx'])[0]).max())
        wl = dict(Qx=d['Qx'], Qy=5, Qz=5, S=d['S'], scheme='upwind2', name=f'sweep instance {k}',
                  params=dict(kn=d['kn'], u_w=d['u_w'], omega=d['omega'], pr=2.0 / 3.0, law='power', dt=dt))
        jobs.append(('steady', wl, 400000))
    t0 = time.perf_counter()
    ctx = mp_.get_context('spawn')
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_job, jobs, chunksize=1)
    sweep = [r for r in res if r['name'].startswith('sweep')]
    return dict(cores=cores, wall_s=time.perf_counter() - t0, jobs=[r for r in res if not r['name'].startswith('sweep')],
                sweep_subset=dict(instances=len(sweep), converged=sum(r['residual'] < 1e-10 for r in sweep),
                                  steps_median=float(np.median([r['steps'] for r in sweep])),
                                  steps_max=max(r['steps'] for r in sweep),
                                  cpu_seconds=sum(r['wall_s'] for r in sweep)))


def cpu_cores():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_baseline(wl, seconds, cores):
    """The oracle (numpy, FP64) on the host: one instance in one process for the one-core
    figure, then `cores` independent instances in as many single-threaded processes for the
    all-core figure (instances are independent, so that is how the host would run a batch).
    Returns pair-updates per second."""
    import multiprocessing as mp_
    pairs = wl['S'] * 2 * wl['Qx'] * wl['Qy'] * wl['Qz']
    n1, t1 = _oracle_worker((wl, 1000, seconds))
    one = pairs * n1 / t1 / 1e9
    ctx = mp_.get_context('spawn')
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(wl, 1000 + b, seconds) for b in range(cores)])
    allc = sum(pairs * n / t for n, t in res) / 1e9
    steps = sum(n for n, _ in res)
    return dict(value=allc, unit='G pair-updates/s', cores=cores, kind='oracle',
                sample=f"{cores} instances (S={wl['S']}, V={pairs // wl['S']}) in {cores} single-threaded processes, "
                       f"{steps} RK3 steps in about {seconds:.0f} s each",
                one_core=dict(value=one, cores=1, sample=f"{n1} RK3 steps of one instance in {t1:.1f} s"))


def main():
    args = parse()
    if args.cpu_suite:
        print(json.dumps({'cpu_suite': cpu_suite(args.cpu_cores or cpu_cores())}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({'error': 'one GPU only: the library drives a single device and has no multi-GPU path',
                          'n_gpus': args.gpus}))
        sys.exit(2)
    import torch
    from paper_1702_01335_amd.workloads import workload
    wl = workload(args.workload)
    own_scheme = args.scheme is None or args.scheme == wl['scheme']
    if args.scheme:
        wl['scheme'] = args.scheme
    device = 'cuda:0'
    torch.cuda.set_device(0)
    q, solver = make_solver(wl, args.batch, device)
    tuned = None
    if args.cells or args.waves:
        c0, w0 = solver.get_launch()
        solver.set_launch(args.cells or c0, args.waves or w0)
    elif not args.no_tune:
        # the library's autotuner times every (node chunk, waves) shape on this state
        c_t, w_t, ms_t = solver.autotune(probe_steps=5, cache_path=args.tune_cache)
        tuned = dict(cells=c_t, waves=w_t, probe_ms_per_step=ms_t if ms_t >= 0 else None,
                     source='timed now' if ms_t >= 0 else args.tune_cache)
    cells, waves = solver.get_launch()
    solver.set_graph(not args.eager)
    pairs = args.batch * wl['S'] * q.V
    ms, wall = time_steps(solver, args.steps, args.warmup)
    value = pairs / (ms * 1e-3) / 1e9

    # per-kernel device time of the same step sequence, HIP events on the solver's stream,
    # per RK3 stage: stage 1 moves 16 B per pair (read F_l, write F1), stages 2 and 3 24 B
    solver.set_timing(True)
    solver.step(min(args.steps, 20))
    tm = solver.get_stage_timing()
    solver.set_timing(False)
    stage_s = [ms / n * 1e-3 for ms, n in zip(tm['stage_ms'], tm['stage_launches'])]
    stage_bytes = [pairs * b for b in STAGE_BYTES]
    stage_avg_s = sum(stage_s) / 3.0
    closure_avg_s = tm['closure_ms'] / tm['closure_launches'] * 1e-3
    bytes_per_launch = pairs * BYTES_PER_PAIR_STEP / 3.0
    achieved = bytes_per_launch / stage_avg_s
    per_stage = [dict(stage=k + 1, avg_launch_us=stage_s[k] * 1e6, bytes_per_launch=stage_bytes[k],
                      achieved=stage_bytes[k] / stage_s[k] / 1e9, frac=stage_bytes[k] / stage_s[k] / HBM_PEAK)
                 for k in range(3)]
    traffic = (profiled_traffic(f"stage_kernel_{args.workload}_b{args.batch}", bytes_per_launch, cells, waves)
               if own_scheme else None)
    res = solver.residual()
    # the stages against what the same GPU gives plain streams of the same mix: the counted
    # bytes of each stage (profiled shape and source only) over its time, against the copy
    # (stage 1) or the add (stages 2 and 3)
    bw_copy, bw_add = delivered_bandwidth(device)
    if traffic:
        for k, ps in enumerate(per_stage):
            cb = traffic['per_stage_bytes'][k]
            ps['counted_bytes'] = cb
            ps['counted_GBs'] = cb / stage_s[k] / 1e9
            ps['frac_of_delivered'] = cb / stage_s[k] / (bw_copy if k == 0 else bw_add)

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # single instance of the same workload (latency-bound; reported for context)
    q1, s1 = make_solver(wl, 1, device)
    s1.set_graph(not args.eager)
    ms1, _ = time_steps(s1, max(args.steps, 50), args.warmup)
    single = dict(batch=1, ms_per_step=ms1, value=wl['S'] * q1.V / (ms1 * 1e-3) / 1e9)
    del s1

    out = {
        'metric': 'G cell-velocity pair-updates/s per RK3 step (% HBM peak)',
        'value': value,
        'unit': 'G pair-updates/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': ms,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64',
        'data': 'synthetic',
        'config': {'workload': f"{args.workload} x {args.batch} independent seeded instances",
                   'batch': args.batch, 'S': wl['S'], 'V': q.V, 'Qx': wl['Qx'], 'Qy': wl['Qy'], 'Qz': wl['Qz'],
                   'scheme': wl['scheme'], 'pairs': pairs,
                   'launch': {'cells': cells, 'waves': waves, 'graph': not args.eager, 'autotuned': tuned},
                   'parallelism': 'single GPU'},
        'hbm_frac_step': pairs * BYTES_PER_PAIR_STEP / (ms * 1e-3) / HBM_PEAK,
        'roofline': {'bound': 'hbm', 'achieved': achieved / 1e9, 'peak': HBM_PEAK / 1e9, 'unit': 'GB/s',
                     'frac': achieved / HBM_PEAK,
                     'traffic': traffic['bytes_per_launch'] if traffic else None, 'traffic_unit': 'bytes/launch',
                     'traffic_detail': traffic,
                     'kernel': 'stage_kernel (the three RK3 stages; frac over their average launch)',
                     'avg_launch_us': stage_avg_s * 1e6, 'bytes_per_launch': bytes_per_launch,
                     'per_stage': per_stage, 'closure_avg_us': closure_avg_s * 1e6,
                     'delivered': {'copy_GBs': bw_copy / 1e9, 'add_GBs': bw_add / 1e9,
                                   'how': 'torch device copy (1 read + 1 write) and add (2 reads + 1 write) '
                                          'of 512 MiB float64 arrays, timed in this run'},
                     'step_frac': pairs * BYTES_PER_PAIR_STEP / (ms * 1e-3) / HBM_PEAK},
        'single_instance': single,
        'residual_max': float(res.max()),
        'wall_s_timed': wall,
    }
    progress(f"step: {value:.2f} G pair-updates/s, stage kernel {stage_avg_s * 1e6:.1f} us")
    if not args.no_sweep or not args.no_warm or not args.no_workloads:
        del solver
        torch.cuda.empty_cache()
    if not args.no_workloads:
        out['workloads'] = workloads_section(min(args.steps, 30), min(args.warmup, 5))
        progress('workloads: ' + ', '.join(f"{w['workload']} x{w['batch']} {w['value']:.2f}" for w in out['workloads']))
    if not args.no_sweep:
        out['sweep'] = sweep_section(args.sweep_instances, args.steady_instances, min(args.steps, 50))
        progress(f"sweep: {out['sweep']['value']:.2f} G pair-updates/s batched")
    if not args.no_warm:
        out['warm_start'] = warm_section(args.warm_train, args.warm_heldout, args.warm_steps)
        progress(f"warm start: wall ratio {out['warm_start']['heldout']['wall_ratio']:.3f}")
    if not args.no_cpu:
        out['cpu_baseline'] = cpu_baseline(wl, args.cpu_seconds, args.cpu_cores or cpu_cores())
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
