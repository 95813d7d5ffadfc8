"""The learned warm start on the neutral plasma ball, trained and judged on separate seeds.

Protocol (the plasma of workloads.c3_plasma, all solves to the same residual 1e-10):
  1. for every training seed, the plasma drawn with that seed from its electrostatic start
     is advanced `steps_per_seed` plain steps (start e^n) while the context records each
     solve's features and target (one interior edge in `stride` per snapshot);
  2. the network is trained on the GPU on all recorded solves (the library's own BF16
     forward/backward kernels and Adam);
  3. for every evaluation seed, four contexts advance the same plasma side by side, the
     solve started from e^n (plain), from the quadratic extrapolation of the last three
     fields, and from the network's prediction, with the energy-optimal line step along
     it and as it is: iterations, the initial residual and the time of the Newmark part
     (right-hand side, start, solve, Faraday; the network's inference is in the start)
     are compared step by step.

A seed's start is carried between contexts through a checkpoint file (the electrostatic
start is computed once per seed).  Prints progress lines and one JSON summary.

    python -m paper_2102_06248_amd.ws_study [--train-seeds 1-10] [--steps-per-seed 500]
        [--eval-seeds 11,12] [--eval-steps 200] [--stride 8] [--epochs 3] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

from . import fepic as F
from . import inputs

E_CHARGE = inputs.ELEMENTARY_CHARGE
M_E = inputs.ELECTRON_MASS


def _seeds(text):
    out = []
    for part in text.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        elif part:
            out.append(int(part))
    return out


def log(*a):
    print(*a, flush=True)


class Plasma:
    """The mesh and species constants of the plasma ball; particles per seed."""

    def __init__(self, n_pairs, n_cells):
        self.n_pairs = n_pairs
        self.xyz, self.tets = inputs.kuhn_cube(n_cells, lo=(-0.04,) * 3, hi=(0.04,) * 3)
        self.m_p = inputs.PROTON_ELECTRON_MASS_RATIO * M_E
        n0 = 2.5e13
        self.w = n0 * (2 * math.pi) ** 1.5 * 0.01 ** 3 / n_pairs
        wpe = math.sqrt(n0 * E_CHARGE ** 2 / (8.8541878128e-12 * M_E))
        self.dt = 0.05 / wpe

    def options(self, warm_start):
        return dict(device=0, precision=0, preconditioner=F.FEPIC_PC_AUX, solve_precision=F.FEPIC_SOLVE_FP64,
                    cg_tol=1e-10, warm_start=warm_start, timing=1)

    def add_species(self, ctx):
        return [F.fepic_add_species(ctx, -E_CHARGE, M_E, self.w), F.fepic_add_species(ctx, E_CHARGE, self.m_p, self.w)]

    def start_file(self, seed, directory):
        """Checkpoint of the seed's plasma at its electrostatic start."""
        x, ue, ui = inputs.gaussian_ball_pairs(self.n_pairs, 0.01, 3.9, 1.0, 0.1, M_E, self.m_p, seed)
        path = os.path.join(directory, f"seed{seed}.ck")
        with F.Simulation(self.xyz, self.tets, **self.options(F.FEPIC_WS_PREV)) as T:
            se, sp = self.add_species(T.ctx)
            F.fepic_upload_particles(T.ctx, se, x, ue)
            F.fepic_upload_particles(T.ctx, sp, x, ui)
            F.fepic_init_electrostatic(T.ctx, 1e-12)
            F.fepic_save(T.ctx, path)
        return path


def _newmark_ms(st):
    return st.ms_rhs + st.ms_warm + st.ms_cg + st.ms_faraday


def run(train_seeds, steps_per_seed, eval_seeds, eval_steps, stride=8, epochs=3, n_pairs=8_000_000, n_cells=55,
        batch=8192, lr=2e-3, workdir=None):
    pl = Plasma(n_pairs, n_cells)
    own_dir = workdir is None
    workdir = workdir or tempfile.mkdtemp(prefix="ws_study_")
    t_start = time.perf_counter()
    log(f"[ws] plasma ball: {len(pl.tets)} tets, {2 * n_pairs} particles; train seeds {train_seeds} x "
        f"{steps_per_seed} steps, eval seeds {eval_seeds} x {eval_steps} steps, stride {stride}")
    R = F.Simulation(pl.xyz, pl.tets, **pl.options(F.FEPIC_WS_PREV))
    P = F.Simulation(pl.xyz, pl.tets, **pl.options(F.FEPIC_WS_PREV))
    X = F.Simulation(pl.xyz, pl.tets, **pl.options(F.FEPIC_WS_EXTRAP2))
    D = F.Simulation(pl.xyz, pl.tets, **pl.options(F.FEPIC_WS_PREV))
    sims = {"plain": P, "extrap2": X, "learned": R, "learned_direct": D}
    try:
        for sim in sims.values():
            pl.add_species(sim.ctx)
        n_snap = len(train_seeds) * steps_per_seed
        recorded_iters = []
        for s in train_seeds:
            path = pl.start_file(s, workdir)
            F.fepic_load(R.ctx, path)
            os.remove(path)
            if not recorded_iters:
                F.fepic_ws_record(R.ctx, stride, n_snap)
            for k in range(steps_per_seed):
                st = F.fepic_step(R.ctx, pl.dt)
                recorded_iters.append(st.cg_iters)
                if k % 100 == 99:
                    log(f"[ws] seed {s}: {k + 1} steps recorded, {st.cg_iters} iterations")
        F.fepic_ws_record(R.ctx, 0)
        n_rec = F.fepic_ws_num_snapshots(R.ctx)
        t0 = time.perf_counter()
        tst = F.fepic_ws_train(R.ctx, epochs=epochs, batch=batch, lr=lr, seed=1, val_fraction=0.1)
        train_s = time.perf_counter() - t0
        log(f"[ws] trained on {n_rec} solves ({tst.n_train_rows} rows, {tst.n_steps} Adam steps) in {train_s:.1f}s: "
            f"train loss {tst.train_loss:.4g}, validation loss {tst.val_loss:.4g}")
        F.fepic_set_warm_start(R.ctx, F.FEPIC_WS_MLP)
        F.fepic_ws_set_weights(D.ctx, F.fepic_ws_get_weights(R.ctx))
        F.fepic_set_warm_start(D.ctx, F.FEPIC_WS_MLP_DIRECT)
        per_seed = []
        for s in eval_seeds:
            path = pl.start_file(s, workdir)
            for sim in sims.values():
                F.fepic_load(sim.ctx, path)
            os.remove(path)
            rows = {name: [] for name in sims}
            for k in range(eval_steps):
                for name, sim in sims.items():
                    t0 = time.perf_counter()
                    st = F.fepic_step(sim.ctx, pl.dt)
                    wall = (time.perf_counter() - t0) * 1e3
                    if st.cg_rel_resid > 1e-10:
                        raise RuntimeError(f"{name} solve stopped at {st.cg_rel_resid:.3g}")
                    rows[name].append((st.cg_iters, st.cg_rel_resid0, _newmark_ms(st), wall))
                if k % 50 == 49:
                    log(f"[ws] eval seed {s}: step {k + 1}, iterations " +
                        ", ".join(f"{name} {r[-1][0]}" for name, r in rows.items()))
            e_p, _, _ = F.fepic_get_fields(P.ctx)
            agree = max(float(np.linalg.norm(F.fepic_get_fields(sim.ctx)[0] - e_p) / np.linalg.norm(e_p))
                        for sim in (R, D))
            summary = {"seed": s, "fields_rel_diff_learned_vs_plain": agree}
            for name, r in rows.items():
                a = np.array(r)
                summary[name] = {"cg_iters": round(float(a[:, 0].mean()), 2), "rel_resid0": float(np.exp(np.log(a[:, 1]).mean())),
                                 "newmark_ms": round(float(a[:, 2].mean()), 3), "step_wall_ms": round(float(a[:, 3].mean()), 3)}
            per_seed.append(summary)
            log(f"[ws] eval seed {s}: {json.dumps(summary)}")
    finally:
        for sim in sims.values():
            sim.close()
        if own_dir:
            try:
                os.rmdir(workdir)
            except OSError:
                pass

    def mean(name, key):
        return round(float(np.mean([p[name][key] for p in per_seed])), 3)

    result = {
        "study": "learned warm start, plasma ball", "tets": int(len(pl.tets)), "particles": 2 * n_pairs,
        "train_seeds": train_seeds, "steps_per_seed": steps_per_seed, "recorded_solves": int(n_rec),
        "row_stride": stride, "train_rows": int(tst.n_train_rows), "adam_steps": int(tst.n_steps), "epochs": epochs,
        "train_loss": tst.train_loss, "val_loss": tst.val_loss, "train_s": round(train_s, 1),
        "recording_cg_iters_mean": round(float(np.mean(recorded_iters)), 2),
        "eval_seeds": eval_seeds, "eval_steps": eval_steps, "per_seed": per_seed,
        "cg_iters": {n: mean(n, "cg_iters") for n in sims},
        "newmark_ms": {n: mean(n, "newmark_ms") for n in sims},
        "step_wall_ms": {n: mean(n, "step_wall_ms") for n in sims},
        "wall_s": round(time.perf_counter() - t_start, 1),
    }
    return result


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-seeds", default="1-10")
    ap.add_argument("--steps-per-seed", type=int, default=500)
    ap.add_argument("--eval-seeds", default="11,12")
    ap.add_argument("--eval-steps", type=int, default=200)
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=8_000_000)
    ap.add_argument("--cells", type=int, default=55)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(_seeds(a.train_seeds), a.steps_per_seed, _seeds(a.eval_seeds), a.eval_steps, a.stride, a.epochs,
              a.pairs, a.cells)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
