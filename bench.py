#!/usr/bin/env python3
"""Benchmark of the FE-PIC hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c5_plasma]

One step = the whole per-step path through the C ABI (fepic_step): sort by tet, field
staging, gather + relativistic Boris + path tracking + Whitney-1 deposit, Newmark
right-hand side, warm start, preconditioned CG to ||b - A e||_2 <= 1e-10 ||b||_2, Faraday.
Inputs are resident on the device before the timed region.  Prints one JSON line.

The headline workload is the refined plasma ball (7,986,000 tets, 64M electrons + 64M
protons), the largest that fits one GPU.  value = particle-steps per second of whole steps
(particles alive at the start of each timed step, summed, over the wall time of the K
steps).  The JSON also carries the particle kernels' own rate and HBM roofline, the
Newmark step time and CG iterations (and the same solve in FP64 arithmetic), the roofline
of the dominant kernel (HIP events on the library's stream over the timed region), the
CPU oracle on a bounded sample (one core and all cores), and shorter runs of the single
electron, the beam and the 998k-tet plasma ball under "workloads".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit) + Newmark step time at CG resid 1e-10"
HBM_PEAK_GBS = 8000.0
FAMILIES = ["push", "stage", "sort", "rhs", "cg_iter", "faraday"]
KERNEL_NAMES = {"push": "k_push+k_cross|k_cross_sparse", "stage": "k_stage", "sort": "k_hist/k_scan/k_scatter", "rhs": "k_rhs",
                "cg_iter": "k_pcg_q<double>+k_pcg_nodes<double>+k_pcg_fold<double>+k_pcg_update<double, 1>",
                "faraday": "k_faraday"}
MIXED_ITER_KERNEL = "k_pcg_q<float>+k_pcg_nodes<float>+k_pcg_fold<float>+k_pcg_update<float, 2>"
JACOBI_ITER_KERNEL = "k_cg_iter"
KERNEL_SOURCES = {"push": "kernels_particles.hip", "stage": "kernels_particles.hip", "sort": "kernels_particles.hip",
                  "rhs": "kernels_fields.hip", "cg_iter": "kernels_fields.hip", "faraday": "kernels_fields.hip"}
EXTRA_DEFAULT = "c1_single_electron,c2_beam,c3_plasma"
# steps, warm-up steps of the shorter runs under "workloads"
EXTRA_STEPS = {"c1_single_electron": (2000, 0), "c2_beam": (20, 5), "c3_plasma": (10, 3), "c5_plasma": (10, 3)}

# The particle step's algorithmic bytes (what the method must move; each word once):
# per particle the state (tet 4 B, three barycentric coordinates and u = gamma v, 4 B each
# in the FP32 path, 8 B in the all-FP64 path) read and written; per occupied tet (per
# species) its 6 edge and 4 face unknowns in FP64 (80), 10 entity ids (40), the gradients
# of the barycentric coordinates in FP32 (48), neighbours (20) and 6 FP64 read-modify-writes
# of the current (96); per face crossing the neighbour's record (68) and 6 more
# read-modify-writes (96).
PUSH_B_PARTICLE = {0: 56, 1: 104}
PUSH_B_TET = 284
PUSH_B_CROSSING = 164


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def push_bytes(n_particles, occupied, crossings, precision=0):
    return PUSH_B_PARTICLE[precision] * n_particles + PUSH_B_TET * occupied + PUSH_B_CROSSING * crossings


def algorithmic_bytes(fam, geo, st, pc="aux", solve="fp64", precision=0):
    """Bytes the method must move per launch (each HBM word once), by kernel family.  A
    "cg_iter" launch is one PCG iteration: one kernel with Jacobi, four with the nodal
    auxiliary-space preconditioner (in FP32 for the inner solves of the mixed form)."""
    n_rows, nnz, ne, nf, nt = geo["n_rows"], geo["nnz"], geo["n_edges"], geo["n_faces"], geo["n_tets"]
    fold = 1 if geo.get("far_levels", 0) > 0 else 0   # the far levels' per-node fold runs
    npart, occ, cross = st["particles"], st["occupied_tets"], st["crossings"]
    if fam == "cg_iter" and pc == "jacobi":   # A values + columns once; per row R, W, S, P and x read
        return 12 * nnz + 80 * n_rows          # and written
    if fam == "cg_iter" and solve == "mixed":
        # the same words in FP32 (values 4 B, (z, p) pairs 8 B, diagonals and Y 16 B per
        # node), column ids, incidences, FP16 edge vectors and ends as before:
        # q 8 nnz + 12 per row; nodes 16 per row, 32 per node; with far levels, their fold:
        # Y read and written per node (32); update 40 read + 16 written per row, 16 per node
        return 8 * nnz + (12 + 16 + 56) * n_rows + 8 * geo["n_int_edges"] + (48 + 32 * fold) * geo["n_aux"]
    if fam == "cg_iter":
        # q = A p: A values + columns, (z, p) read, q written: 12 nnz + 24 per row;
        # nodes: one 4 B incidence per interior edge end, r, q and the FP16 edge vector per
        # row (24), scale read and Y written per node (64); with far levels, their fold: Y
        # read and written per node (64);
        # update: r, q, z, p, x, 1/A_jj, edge vector, ends read (64) and r, z, p, x written
        # (32) per row, Y read per node (32)
        return 12 * nnz + (24 + 24 + 96) * n_rows + 8 * geo["n_int_edges"] + (96 + 64 * fold) * geo["n_aux"]
    if fam == "rhs":          # M, S values + columns; e, e_prev, dG_new, dG_old read; b written
        return 20 * nnz + 40 * n_rows
    if fam == "push":         # all species of one step
        return push_bytes(npart, occ, cross, precision)
    if fam == "stage":        # per tet record write (9 x 4 B); e, b once; grad 72 B + 10 ids
        return nt * (36 + 72 + 40) + 8 * (ne + nf)
    if fam == "faraday":      # 3 edge ids + b read/write per face; e^{n+1}, e^n once
        return nf * (12 + 16) + 16 * ne
    if fam == "sort":         # histogram read of tet; scatter read + write of 36 B payload
        return npart * (4 + 72) + 12 * nt
    return 0


def source_hash(fam):
    p = os.path.join(ROOT, "paper_2102_06248_amd", "csrc", KERNEL_SOURCES[fam])
    return hashlib.sha1(open(p, "rb").read()).hexdigest()[:12]


def profile_key(fam, pc, solve="fp64"):
    """Name stem of a family's counter summary under profiles/."""
    if fam == "cg_iter" and pc == "jacobi":
        return "cg_iter_jacobi"
    if fam == "cg_iter" and solve == "mixed":
        return "cg_iter_mixed"
    return fam


def traffic_from_profile(fam, workload, pc="aux", solve="fp64"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; None otherwise."""
    p = os.path.join(ROOT, "profiles", f"{profile_key(fam, pc, solve)}_{workload}_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_sha1") != source_hash(fam):
        return None
    return d.get("hbm_bytes_per_launch")


def worker_count():
    """Threads for the all-cores oracle timing: the CPUs this process may run on, at most
    16 (one GPU's share of a GPU host's cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


# ---------------------------------------------------------------------- CPU oracle legs

def cpu_push_sample(wl, n_sample=1_000_000, target_s=10.0, max_steps=40):
    """The oracle's particle step (gather, Boris, walk, deposit: oracle/particles.c) on the
    first n_sample particles of the workload's seeded draw (split evenly over the species),
    in the workload's initial fields: zero for the co-located neutral pairs of the plasma
    balls (their charge density, and so the electrostatic start, is zero).  Timed on one
    thread for about target_s seconds, then on worker_count() threads, each pushing a
    contiguous chunk into its own current vector (ctypes releases the GIL), over the same
    number of steps."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import particles as op
    from oracle.mesh import Mesh

    t0 = time.perf_counter()
    m = Mesh(wl["xyz"], wl["tets"])
    cm = op.CMesh(m)
    per = n_sample // len(wl["species"])
    x0 = wl["species"][0]["x"][:per]
    tet0 = m.locate(x0)
    same_x = all(np.array_equal(s["x"][:per], x0) for s in wl["species"])
    log(f"[bench] oracle set-up for the CPU baseline: {time.perf_counter() - t0:.1f} s")
    e, b = np.zeros(m.n_edges), np.zeros(m.n_faces)
    if wl.get("B0") is not None:
        b = m.face_dofs_of_uniform_field(wl["B0"])
    state = []
    for s in wl["species"]:
        tet = tet0 if same_x else m.locate(s["x"][:per])
        keep = tet >= 0
        state.append(dict(q=s["q"], m=s["m"], w=s["w"], x=np.ascontiguousarray(s["x"][:per][keep]),
                          u=np.ascontiguousarray(s["u"][:per][keep], dtype=np.float64),
                          tet=tet[keep].astype(np.int64), alive=np.ones(int(keep.sum()), np.int8)))
    n_total = sum(len(s["x"]) for s in state)

    def one_step(chunks, dg, pool):
        # each chunk deposits into its own current vector (allocated once, outside the timing)
        def work(k):
            j, lo, hi = chunks[k]
            s = state[j]
            rc, _ = op.push(cm, s["x"][lo:hi], s["u"][lo:hi], s["tet"][lo:hi], s["alive"][lo:hi], s["q"], s["m"],
                            s["w"], wl["dt"], e, b, dg[k])
            return rc

        if pool is None:
            for k in range(len(chunks)):
                work(k)
        else:
            list(pool.map(work, range(len(chunks))))

    def slices(n_threads):
        out = []
        for j, s in enumerate(state):
            n = len(s["x"])
            edges = np.linspace(0, n, n_threads + 1).astype(int)
            out += [(j, int(edges[i]), int(edges[i + 1])) for i in range(n_threads)]
        return out

    def alive_count():
        return sum(int(s["alive"].sum()) for s in state)

    one = [(j, 0, len(s["x"])) for j, s in enumerate(state)]
    dg1 = [np.zeros(m.n_edges) for _ in one]
    psteps1, steps1, t1 = 0, 0, 0.0
    while steps1 < max_steps and (t1 < target_s or steps1 < 2):
        n_live = alive_count()
        t = time.perf_counter()
        one_step(one, dg1, None)
        t1 += time.perf_counter() - t
        psteps1 += n_live
        steps1 += 1
    nw = worker_count()
    chunks = slices(nw)
    dgn = [np.zeros(m.n_edges) for _ in chunks]
    psteps_n, tn = 0, 0.0
    with ThreadPoolExecutor(max_workers=nw) as pool:
        for _ in range(steps1):
            n_live = alive_count()
            t = time.perf_counter()
            one_step(chunks, dgn, pool)
            tn += time.perf_counter() - t
            psteps_n += n_live
    sample = (f"particle step (gather, Boris, walk, deposit) of the first {n_total} particles of the workload's "
              f"seeded draw ({len(state)} species) in its initial fields, {steps1} steps on one thread "
              f"({t1:.1f} s), then the same number of steps on {nw} threads ({tn:.1f} s); field solve not timed")
    return {"value": psteps_n / tn, "unit": "particle-steps/s", "cores": nw, "kind": "oracle", "sample": sample,
            "os_cpu_count": os.cpu_count(), "seconds": round(tn, 2),
            "single_core": {"value": psteps1 / t1, "cores": 1, "seconds": round(t1, 2), "steps": steps1}}


def cpu_full_steps(wl, n_steps=12):
    """The oracle's whole step (particle push + Newmark Jacobi-PCG + Faraday) on the same
    workload from its own electrostatic start, single thread (numpy/scipy thread pools
    limited to 1)."""
    from threadpoolctl import threadpool_limits

    from oracle.pic import OracleSim

    with threadpool_limits(limits=1):
        osim = OracleSim(wl["xyz"], wl["tets"])
        n_total = 0
        for sp in wl["species"]:
            s = osim.add_species(sp["q"], sp["m"], sp["w"])
            osim.upload_particles(s, sp["x"], sp["u"])
            n_total += len(sp["x"])
        if wl.get("B0") is not None:
            osim.set_uniform_B(wl["B0"])
        osim.init_electrostatic(tol=1e-12)
        t_all, t_field, iters, psteps = 0.0, 0.0, [], 0
        for _ in range(n_steps):
            n_live = sum(int(sp_.alive.sum()) for sp_ in osim.species)
            t0 = time.perf_counter()
            st = osim.step(wl["dt"], wl["beta"], wl["gamma"])
            t_all += time.perf_counter() - t0
            iters.append(st["cg_iters"])
            psteps += n_live
    return {"value": psteps / t_all, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"{n_steps} full steps of the same workload ({n_total} particles, no injection) from the "
                       f"oracle's own electrostatic start: {t_all:.1f} s, Newmark Jacobi-PCG "
                       f"{np.mean(iters):.0f} iterations per step; single thread"),
            "newmark_cg_iters_mean": float(np.mean(iters)), "seconds": round(t_all, 2),
            "ms_per_step": round(1e3 * t_all / n_steps, 2)}


def cpu_baseline(wl, n_sample=None):
    if wl["name"] in ("c3_plasma", "c5_plasma"):
        return cpu_push_sample(wl, n_sample or 1_000_000)
    if wl["name"] == "c1_single_electron":
        return cpu_full_steps(wl, n_steps=wl["steps"])
    return cpu_full_steps(wl)


# ---------------------------------------------------------------------- Adams-Bashforth

def ab_bytes_per_particle_step(k):
    """Algorithmic HBM bytes of one Adams-Bashforth-k particle step: the particle state read
    and written (tet 4 B, three barycentric coordinates and the velocity in FP64: 52 B each
    way), the history it needs (positions r^n..r^{n+1-k}, velocities v^{n-1}..v^{n+1-k},
    accelerations a^{n-1}..a^{n+1-k}: 3 (3k - 2) doubles) and the three new levels it must
    keep (r^{n+1}, v^{n+1}, a^n: 9 doubles)."""
    return 2 * 52 + 8 * 3 * (3 * k - 2) + 8 * 9


def ab_bench(args, F, torch, sim, wl, species):
    """Particle-only Adams-Bashforth pushes of every species in the workload's initial
    fields (electrostatic start, fields frozen): fepic_push_particles with the pusher option
    set to Adams-Bashforth.
    Prints one JSON line; the roofline is the AB kernel's, HIP-event timed."""
    ctx = sim.ctx
    k_ord, dt = args.ab_order, wl["dt"]
    warmup = max(args.warmup, k_ord)              # the history reaches the full order first
    for k in range(warmup):
        st = F.fepic_push_particles(ctx, dt)
        log(f"[bench] ab warmup {k}: {st.n_particles} particles, {st.n_crossings} crossings")
    sizes = F.fepic_get_topology_sizes(ctx)
    F.fepic_kernel_timing(ctx, "push", 1 + args.steps * 4 * len(species))
    n_live = sum(F.fepic_num_particles(ctx, s) for s in species)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psteps, cross = 0, 0
    for k in range(args.steps):
        st = F.fepic_push_particles(ctx, dt)
        psteps += n_live
        n_live = st.n_particles
        cross += st.n_crossings
        log(f"[bench] ab step {k}: {n_live} particles, {st.n_crossings} crossings")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, nl = F.fepic_kernel_time(ctx, "push")
    kernel_s = ms / 1e3
    if args.copy_calibration:
        copy_calibration(torch)
    per_ps = ab_bytes_per_particle_step(k_ord)
    # per launch: the particles' bytes, one staged record per tet (128 B) and the current
    # vector written once
    total_bytes = psteps * per_ps + nl * (128 * len(wl["tets"]) + 8 * sizes["n_edges"])
    achieved = total_bytes / kernel_s / 1e9
    traffic = None
    cpath = os.path.join(ROOT, "profiles", f"push_ab{k_ord}_{wl['name']}_counters.json")
    if os.path.exists(cpath):
        cd = json.load(open(cpath))
        src = os.path.join(ROOT, "paper_2102_06248_amd", "csrc", cd["source"])
        if cd.get("source_sha1") == hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]:
            traffic = cd["hbm_bytes_per_launch"]
    out = {
        "metric": "particle-steps/s (Adams-Bashforth gather+push+curved walk+deposit, fields frozen)",
        "value": psteps / elapsed, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "tets": len(wl["tets"]), "particles": sum(len(s["x"]) for s in wl["species"]),
                   "mean_live_particles": round(psteps / args.steps), "dt": dt, "ab_order": k_ord,
                   "fields": "electrostatic start, frozen", "parallelism": "single GPU"},
        "kernel_particle_steps_per_s": psteps / kernel_s,
        "crossings_per_particle_step": round(cross / psteps, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_push_ab",
                     "avg_launch_us": round(kernel_s / nl * 1e6, 3), "launches": nl,
                     "algorithmic_bytes_per_particle_step": per_ps,
                     "algorithmic_bytes_per_launch": int(total_bytes / nl)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    sim.close()


def copy_calibration(torch):
    """A plain 256 MiB device copy (the counter passes calibrate FETCH_SIZE and WRITE_SIZE
    against it)."""
    a = torch.empty(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


# ---------------------------------------------------------------------- Boris whole steps

def run_workload(args, F, torch, name, steps, warmup, with_cpu, with_fp64_solve):
    """Builds the workload, runs `warmup` untimed and `steps` timed whole steps, and returns
    the measurements as a dict (the headline JSON's fields)."""
    from paper_2102_06248_amd import workloads

    kw = {}
    if args.particles and name == args.workload:
        kw = {"n_particles": args.particles} if name == "c2_beam" else {"n_pairs": args.particles}
    t0 = time.perf_counter()
    wl = workloads.WORKLOADS[name](**kw)
    log(f"[bench] workload {name} built in {time.perf_counter() - t0:.1f}s: "
        f"{len(wl['tets'])} tets, {sum(len(s['x']) for s in wl['species'])} particles")
    headline = name == args.workload
    warm = (args.warm_start if headline else None) or wl.get("warm_start", "prev")
    ws = {"prev": F.FEPIC_WS_PREV, "extrap1": F.FEPIC_WS_EXTRAP1, "extrap2": F.FEPIC_WS_EXTRAP2,
          "mlp": F.FEPIC_WS_PREV}[warm]
    precision = {"auto": wl["precision"], "fp32": 0, "fp64": 1}[args.precision if headline else "auto"]
    ab_pusher = headline and args.pusher == "ab"
    if ab_pusher:
        precision = 1                      # the Adams-Bashforth pusher is FP64 only
    pc = args.preconditioner if headline else "aux"
    solve = (args.solve if headline else None) or (wl.get("solve", "fp64") if pc == "aux" else "fp64")
    if solve == "mixed" and pc != "aux":
        raise SystemExit("--solve mixed needs --preconditioner aux")
    inner_tol = (args.inner_tol if headline else None) or wl.get("inner_tol")
    sort_period = args.sort_period if (headline and args.sort_period is not None) else wl.get("sort_period", 1)
    sim = F.Simulation(wl["xyz"], wl["tets"], device=0, precision=precision, warm_start=ws,
                       sort_period=sort_period, timing=1, diagnostics=1 if args.diagnostics else 0,
                       preconditioner=F.FEPIC_PC_AUX if pc == "aux" else F.FEPIC_PC_JACOBI,
                       solve_precision=F.FEPIC_SOLVE_MIXED if solve == "mixed" else F.FEPIC_SOLVE_FP64,
                       **({"mixed_inner_tol": inner_tol} if (solve == "mixed" and inner_tol) else {}),
                       walk={"auto": F.FEPIC_WALK_AUTO, "queue": F.FEPIC_WALK_QUEUE,
                             "fused": F.FEPIC_WALK_FUSED}[args.walk if headline else "auto"],
                       pusher=F.FEPIC_PUSHER_AB if ab_pusher else F.FEPIC_PUSHER_BORIS,
                       ab_order=args.ab_order if ab_pusher else 4)
    ctx = sim.ctx
    species = []
    for sp in wl["species"]:
        s = F.fepic_add_species(ctx, sp["q"], sp["m"], sp["w"])
        rej = F.fepic_upload_particles(ctx, s, sp["x"], sp["u"])
        species.append(s)
        log(f"[bench] species {s}: {len(sp['x'])} uploaded, {rej} rejected")
    if wl.get("B0") is not None:
        F.fepic_set_uniform_B(ctx, wl["B0"])
    it = F.fepic_init_electrostatic(ctx, 1e-12)
    log(f"[bench] electrostatic start: {it} CG iterations")
    if ab_pusher:
        ab_bench(args, F, torch, sim, wl, species)
        return None
    inject = args.inject and wl.get("inject_per_step")
    n_train = args.train_steps if (headline and warm == "mlp") else 0
    batches = ([workloads.c2_injection_batch(k) for k in range(n_train + warmup + steps)] if inject else [])
    next_id = [10 ** 9]
    staged = []
    if inject and args.inject_from == "device":
        # every batch resident in HBM before any step runs
        for k, (x, u) in enumerate(batches):
            ids = np.arange(10 ** 9 + k * len(x), 10 ** 9 + (k + 1) * len(x), dtype=np.int64)
            staged.append([torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in (x, u, ids)])
        torch.cuda.synchronize()

    def one_step(k):
        if inject:
            x, u = batches[k]
            if staged:
                dx, du, did = staged[k]
                F.fepic_inject_particles_device(ctx, species[0], len(x), dx.data_ptr(), du.data_ptr(), did.data_ptr())
            else:
                ids = np.arange(next_id[0], next_id[0] + len(x))
                F.fepic_inject_particles(ctx, species[0], x, u, ids=ids)
            next_id[0] += len(x)
        return F.fepic_step(ctx, wl["dt"], wl["beta"], wl["gamma"])

    learned = None
    if n_train:
        # learned warm start: record plain solves, train on the GPU, then solve from the network
        F.fepic_ws_record(ctx, 1, n_train)
        plain_iters = []
        for k in range(n_train):
            st = one_step(k)
            plain_iters.append(st.cg_iters)
        F.fepic_ws_record(ctx, 0)
        tst = F.fepic_ws_train(ctx, epochs=6, batch=8192, lr=2e-3, seed=1, val_fraction=0.25)
        F.fepic_set_warm_start(ctx, F.FEPIC_WS_MLP)
        learned = {"train_steps": n_train, "plain_cg_iters_mean_while_recording": round(float(np.mean(plain_iters)), 2),
                   "train": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in tst.as_dict().items()}}
        log(f"[bench] trained the warm-start network on {n_train} solves: {learned['train']}")
    warm_st = None    # the last warm-up step's statistics (None without warm-up steps)
    for k in range(warmup):
        st = warm_st = one_step(n_train + k)
        if k < 5 or k == warmup - 1:
            log(f"[bench] warmup {k}: cg {st.cg_iters} iters, {st.n_particles} particles, {st.n_crossings} crossings")
    # geometry of the work, for algorithmic bytes
    sizes = F.fepic_get_topology_sizes(ctx)
    nnz_int = F.fepic_get_matrix_nnz(ctx, 0)
    geo = {"n_rows": sizes["n_edges"], "nnz": nnz_int + (sizes["n_edges"] - sizes["n_int_edges"]),
           "n_edges": sizes["n_edges"], "n_faces": sizes["n_faces"], "n_tets": len(wl["tets"]),
           "n_int_edges": sizes["n_int_edges"], "n_aux": sizes["n_int_nodes"],
           "far_levels": max(0, int(warm_st.pc_far_levels)) if warm_st is not None else 0}
    occ = 0     # tets holding particles, counted per species (each species' launch reads them)
    for s in species:
        occ += len(np.unique(F.fepic_get_particles(ctx, s, fields=("tet",))["tet"]))
    for fam in FAMILIES:
        F.fepic_kernel_timing(ctx, fam, 1 + steps * (1200 if fam.startswith("cg") else 4))

    n_start = sum(F.fepic_num_particles(ctx, s) for s in species)   # live particles before the first timed step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psteps, cg_iters, cross, newmark_ms, push_ms, stats = 0, [], 0, [], [], []
    for k in range(steps):
        n_before = n_start if k == 0 else stats[-1].n_particles
        if inject:
            n_before += len(batches[n_train + warmup + k][0])
        st = one_step(n_train + warmup + k)
        psteps += n_before
        cg_iters.append(st.cg_iters)
        cross += st.n_crossings
        newmark_ms.append(st.ms_rhs + st.ms_warm + st.ms_cg + st.ms_faraday)
        push_ms.append(st.ms_stage + st.ms_particles)
        stats.append(st)
        if steps <= 50 or k % (steps // 20) == 0 or k == steps - 1:
            diag = (f", continuity {st.cont_resid_rel:.2e}, gauss drift {st.gauss_drift_check_rel:.2e}"
                    if args.diagnostics else "")
            log(f"[bench] {name} step {k}: cg {st.cg_iters} iters, {st.n_particles} particles, "
                f"{st.n_crossings} crossings, push {push_ms[-1]:.3f} ms, newmark {newmark_ms[-1]:.3f} ms{diag}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    fam_time = {}
    for fam in FAMILIES:
        ms, n = F.fepic_kernel_time(ctx, fam)
        fam_time[fam] = (ms, n)
        F.fepic_kernel_timing(ctx, fam, 0)
    mean_particles = psteps / steps
    wst = {"particles": mean_particles, "occupied_tets": occ, "crossings": cross / steps}

    # dominant kernel family over the timed region
    dominant = max(fam_time, key=lambda f: fam_time[f][0])
    ms_tot, nl = fam_time[dominant]
    work_share = 1.0
    if dominant == "push":
        per_launch = algorithmic_bytes("push", geo, wst, precision=precision) * steps / max(nl, 1)
    else:
        per_launch = algorithmic_bytes(dominant, geo, wst, pc, solve, precision)
    if dominant == "cg_iter":
        # launches that find the solve converged move nothing: average the algorithmic
        # bytes over all launches (iterations / launches of a full iteration's bytes)
        work_share = min(1.0, sum(cg_iters) / nl)
    avg_s = ms_tot / nl / 1e3
    achieved = per_launch * work_share / avg_s / 1e9
    traffic = traffic_from_profile(dominant, name, pc, solve)
    if traffic is not None:
        traffic = int(traffic * work_share)   # counters are per working launch (median)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": (JACOBI_ITER_KERNEL if pc == "jacobi" else MIXED_ITER_KERNEL if solve == "mixed"
                           else KERNEL_NAMES[dominant]) if dominant == "cg_iter" else KERNEL_NAMES[dominant],
                "avg_launch_us": round(avg_s * 1e6, 3), "launches": nl,
                "working_launch_share": round(work_share, 4),
                "algorithmic_bytes_per_launch": int(per_launch * work_share)}

    # the particle kernels' own roofline: one launch = one species' k_push (+ k_cross)
    pms, pn = fam_time["push"]
    pbytes = algorithmic_bytes("push", geo, wst, precision=precision)
    ptraffic = traffic_from_profile("push", name)
    roof_p = None
    if pms > 0:
        ach_p = pbytes * steps / (pms / 1e3) / 1e9
        roof_p = {"bound": "hbm", "achieved": round(ach_p, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(ach_p / HBM_PEAK_GBS, 4), "traffic": ptraffic, "kernel": KERNEL_NAMES["push"],
                  "avg_launch_us": round(pms / max(pn, 1) * 1e3, 3), "launches": pn,
                  "algorithmic_bytes_per_launch": int(pbytes * steps / max(pn, 1)),
                  "bytes_model": {"per_particle": PUSH_B_PARTICLE[precision], "per_occupied_tet": PUSH_B_TET,
                                  "per_crossing": PUSH_B_CROSSING,
                                  "particles_per_step": round(mean_particles),
                                  "occupied_tets_per_step": occ, "crossings_per_step": round(cross / steps)}}
    sms, tms = fam_time["stage"][0], fam_time["sort"][0]
    psteps_all = mean_particles * steps
    push_info = {"particle_steps_per_s": psteps_all / (pms / 1e3) if pms > 0 else None,
                 "with_staging": psteps_all / ((pms + sms) / 1e3) if pms > 0 else None,
                 "with_staging_and_sort": psteps_all / ((pms + sms + tms) / 1e3) if pms > 0 else None,
                 "ms_per_step": round(pms / steps, 4)}
    breakdown = {f: {"ms_per_step": round(fam_time[f][0] / steps, 4), "launches_per_step": fam_time[f][1] / steps}
                 for f in FAMILIES}
    n_total = sum(len(s["x"]) for s in wl["species"])
    out = {
        "value": psteps / elapsed, "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * elapsed / steps,
        "dtype": "f32+f64" if precision == 0 else "f64",
        "config": {"workload": wl["name"], "tets": len(wl["tets"]), "particles": n_total,
                   "mean_live_particles": round(mean_particles), "dt": wl["dt"], "beta": wl["beta"],
                   "gamma": wl["gamma"], "cg_tol": 1e-10, "preconditioner": pc, "solve": solve,
                   "mixed_inner_tol": (inner_tol or 1e-4) if solve == "mixed" else None,
                   "walk": args.walk if headline else "auto", "warm_start": warm,
                   "sort_period": "auto" if sort_period == F.FEPIC_SORT_AUTO else sort_period,
                   "inject_per_step": int(wl.get("inject_per_step") or 0) if inject else 0,
                   "inject_from": args.inject_from if inject else None,
                   "precision": ("fp32 push / fp64 deposit" if precision == 0 else "all fp64 particles")
                   + (" / fp64 residuals around fp32 inner solves" if solve == "mixed" else " / fp64 solve"),
                   "diagnostics_in_timed_steps": bool(args.diagnostics), "parallelism": "single GPU"},
        "newmark_ms_per_step": round(float(np.mean(newmark_ms)), 4),
        "cg_iters_mean": round(float(np.mean(cg_iters)), 2),
        "cg_passes_mean": round(float(np.mean([st.cg_passes for st in stats])), 2),
        "push": push_info,
        "crossings_per_particle_step": round(cross / psteps, 4),
        "kernel_breakdown": breakdown,
        "roofline": roofline,
        "roofline_particles": roof_p,
    }
    if learned is not None:
        learned["mlp_cg_iters_mean"] = out["cg_iters_mean"]
        out["learned_warm_start"] = learned
    if args.diagnostics:
        out["conservation"] = {
            "cont_resid_rel_max": max(st.cont_resid_rel for st in stats),
            "gauss_drift_check_rel_max": max(st.gauss_drift_check_rel for st in stats),
            "gauss_resid_rel_max": max(st.gauss_resid_rel for st in stats)}
    if with_fp64_solve and solve == "mixed":
        # the same Newmark solve in FP64 arithmetic (FP64 PCG, same preconditioner and
        # stopping rule), on the steps after the timed region
        F.fepic_set_solve_precision(ctx, F.FEPIC_SOLVE_FP64)
        ms64, it64 = [], []
        for k in range(3):
            st = one_step(n_train + warmup + steps + k) if not inject else None
            if st is None:
                break
            ms64.append(st.ms_rhs + st.ms_warm + st.ms_cg + st.ms_faraday)
            it64.append(st.cg_iters)
        if ms64:
            out["newmark_fp64_solve"] = {"ms_per_step": round(float(np.mean(ms64[1:] or ms64)), 4),
                                         "cg_iters_mean": round(float(np.mean(it64[1:] or it64)), 2),
                                         "steps": len(ms64[1:] or ms64),
                                         "note": "FP64 PCG with the same preconditioner and tolerance, timed on "
                                                 "the steps after the timed region (first one discarded)"}
    if args.copy_calibration and headline:
        copy_calibration(torch)
    sim.close()
    if with_cpu:
        log(f"[bench] timing the CPU oracle on a bounded sample of {name}")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample if headline else None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5_plasma", choices=["c2_beam", "c3_plasma", "c5_plasma"])
    ap.add_argument("--extra-workloads", default=EXTRA_DEFAULT,
                    help="comma-separated workloads also run (shorter) and reported under 'workloads'; "
                         "'none' for none")
    ap.add_argument("--particles", type=int, default=None, help="override the particle count (pairs for plasmas)")
    ap.add_argument("--precision", default="auto", choices=["auto", "fp32", "fp64"],
                    help="particle path precision (auto: the workload's; fp64 = all-FP64 path)")
    ap.add_argument("--warm-start", default=None, choices=["prev", "extrap1", "extrap2", "mlp"],
                    help="start of the Newmark solve (default: the workload's, else the previous field)")
    ap.add_argument("--train-steps", type=int, default=40,
                    help="mlp: plain steps recorded for training before the warm-up steps")
    ap.add_argument("--diagnostics", action="store_true",
                    help="run the conservation diagnostics every step (continuity, Gauss drift)")
    ap.add_argument("--sort-period", type=int, default=None,
                    help="re-sort particles by tet every this many steps; -1: each species when a 64th "
                         "of it has left its tet (default: the workload's)")
    ap.add_argument("--walk", default="auto", choices=["auto", "queue", "fused"],
                    help="crossing paths: chosen from the last step's crossings, queue + second kernel, or in place")
    ap.add_argument("--solve", default=None, choices=["fp64", "mixed"],
                    help="Newmark solve arithmetic: FP64 PCG, or FP64 residuals around FP32 inner PCG "
                         "(auxiliary-space preconditioner only); default: the workload's")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="--solve mixed: residual reduction of one FP32 pass (default: the workload's)")
    ap.add_argument("--preconditioner", default="aux", choices=["aux", "jacobi"],
                    help="Newmark PCG preconditioner: nodal auxiliary space (default) or Jacobi")
    ap.add_argument("--inject", type=int, default=1, help="inject the beam's per-step batch (c2)")
    ap.add_argument("--inject-from", default="device", choices=["device", "host"],
                    help="device: batches staged in HBM before the timed region; host: copied per step")
    ap.add_argument("--cpu-sample", type=int, default=None, help="limit the oracle's particle count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pusher", default="boris", choices=["boris", "ab"],
                    help="ab: time particle-only Adams-Bashforth pushes instead of whole steps")
    ap.add_argument("--ab-order", type=int, default=4, help="order of the Adams-Bashforth pusher (1..5)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; a mesh-partition "
              "sharding is described in the design notes but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2102_06248_amd import fepic as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    head = run_workload(args, F, torch, args.workload, args.steps, args.warmup,
                        with_cpu=not args.no_cpu_baseline, with_fp64_solve=True)
    if head is None:          # --pusher ab printed its own line
        return
    extras = {}
    names = [] if args.extra_workloads in ("", "none") else args.extra_workloads.split(",")
    if args.pusher == "boris" and args.warm_start != "mlp":
        for name in names:
            if name == args.workload:
                continue
            if name == "c1_single_electron":
                extras[name] = run_c1(F, torch, with_cpu=not args.no_cpu_baseline)
                continue
            st, wu = EXTRA_STEPS[name]
            r = run_workload(args, F, torch, name, st, wu, with_cpu=not args.no_cpu_baseline, with_fp64_solve=False)
            extras[name] = {k: r[k] for k in ("value", "ms_per_step", "steps", "warmup", "newmark_ms_per_step",
                                              "cg_iters_mean", "cg_passes_mean", "push", "roofline",
                                              "roofline_particles", "crossings_per_particle_step", "config")}
            extras[name]["cpu_baseline"] = r.get("cpu_baseline")
    out = {
        "metric": METRIC, "value": head["value"], "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": head["dtype"],
        "data": "synthetic",
    }
    for k, v in head.items():
        if k not in out and k not in ("steps", "warmup"):
            out[k] = v
    out.setdefault("cpu_baseline", None)
    out["workloads"] = extras
    print(json.dumps(out), flush=True)


def run_c1(F, torch, with_cpu):
    """The single electron in a uniform B (1,296 tets, all FP64, Jacobi-PCG, 2000 steps):
    a latency-bound workload, timed whole (no warm-up), with the oracle's 2000 steps."""
    from paper_2102_06248_amd import workloads

    wl = workloads.c1_single_electron()
    sim = F.Simulation(wl["xyz"], wl["tets"], device=0, precision=F.FEPIC_ALL_FP64, timing=1,
                       preconditioner=F.FEPIC_PC_JACOBI, solve_precision=F.FEPIC_SOLVE_FP64)
    ctx = sim.ctx
    sp = wl["species"][0]
    s = F.fepic_add_species(ctx, sp["q"], sp["m"], sp["w"])
    F.fepic_upload_particles(ctx, s, sp["x"], sp["u"])
    F.fepic_set_uniform_B(ctx, wl["B0"])
    F.fepic_init_electrostatic(ctx, 1e-14)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, nm = [], []
    for _ in range(wl["steps"]):
        st = F.fepic_step(ctx, wl["dt"], wl["beta"], wl["gamma"])
        iters.append(st.cg_iters)
        nm.append(st.ms_rhs + st.ms_warm + st.ms_cg + st.ms_faraday)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.close()
    log(f"[bench] c1_single_electron: {wl['steps']} steps in {el:.2f} s")
    out = {"value": wl["steps"] / el, "ms_per_step": 1e3 * el / wl["steps"], "steps": wl["steps"], "warmup": 0,
           "newmark_ms_per_step": round(float(np.mean(nm)), 4), "cg_iters_mean": round(float(np.mean(iters)), 2),
           "config": {"workload": wl["name"], "tets": len(wl["tets"]), "particles": 1, "dt": wl["dt"],
                      "precision": "all fp64, Jacobi-PCG", "note": "latency-bound: one particle, 1,854 edges"}}
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    return out


if __name__ == "__main__":
    main()
