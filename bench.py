#!/usr/bin/env python3
"""Throughput benchmark of the HWENO-GR hot path on one MI355X.

Workload: the 2D viscous shock tube on [0,1] x [0,0.5] with 1000 x 500
cells (gamma 1.4, Re 200, Pr 0.73, adiabatic no-slip walls at x = 0, x = 1,
y = 0 and a symmetry line at y = 0.5; rho = 120 | 1.2, p = rho/gamma, at rest),
advanced by SSP-RK3 steps with the paper's time-step rule from t = 0.
A step is three stages; each stage is one full residual evaluation (ghost
fill, characteristic HWENO reconstruction with the positivity limiter, weak
derivative moments, gradient reconstruction, fluxes) plus the stage update.
The state lives in HBM before the timed region starts.

Prints one JSON line.  ``value`` = cell-stage updates per second.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = '2D cell-stage updates/s FP64 + %HBM roofline; batched & adjoint vs plain'
UNIT = 'cell-stage updates/s'
NX, NY = 1000, 500
EXTENT = (0.0, 1.0, 0.0, 0.5)
BCS = ('noslip', 'noslip', 'noslip', 'slip')
PHYS = dict(gamma=1.4, Pr=0.73, mu_ref=1.0 / 200.0)

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6        # FP64 vector (FP64 matrix is the same)
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 operations per cell (per face for 'flux') of each kernel
# class, counted from the operations of the method as the kernels perform
# them once per cell (additions, multiplications, divisions, square roots
# each one flop; a fused multiply-add two):
#   recon: 8 scalar reconstructions (projection 136, quartic candidate 138,
#          smoothness indicator 87, weights 45, combination 35, 15 point values
#          135, moment 5) = 4648; characteristic bases 75; back-transform 1024;
#          limiter on 30 points 420; wbar 240; wave speed 300.
#   grad:  6 scalar reconstructions at 21 points (495 each) = 2970; volume
#          fluxes at 18 points 792.
#   rbar:  interface averages, face moments, 18 weak moments.
#   flux:  per face 6 point fluxes and PP speed bounds, 12 LF combinations.
#   update: assembly of 12 residual entries and the stage combination.
FLOPS = {'recon': 6707, 'grad': 3762, 'rbar': 414, 'flux': 560, 'update': 400}
# Algorithmic HBM bytes per cell-stage of the whole path if every input were
# read once and every output written once (stage average: 256 B residual
# in/out + the RK bases of stages 2 and 3).
ALGO_BYTES_PER_CELL_STAGE = 277.0


def units_per_launch(kind):
    if kind == 'recon':
        return (NX + 6) * (NY + 6)
    if kind == 'rbar':
        return (NX + 4) * (NY + 4)
    if kind == 'grad':
        return (NX + 2) * (NY + 2)
    if kind == 'flux':
        return (NX + 1) * NY + NX * (NY + 1)
    return NX * NY


def cpu_baseline(rows=64):
    """The oracle on a bounded sample: three stage residual evaluations (one
    RK3 step's spatial work) on a 1000 x ``rows`` window of the same grid,
    with its true neighbours as halo, on one thread."""
    from threadpoolctl import threadpool_limits
    from oracle.common import Options, Physics
    from oracle.scheme2d import Scheme2D
    from paper_2608_10569_amd import workloads
    U = workloads.viscous_shock_tube_2d(NX, NY)
    sc = Scheme2D(NX, NY, *EXTENT, Physics(**PHYS), Options(cfl=0.3), bc=BCS)
    Ug = sc.ghost(U)
    j0 = (NY - rows) // 2
    W = Ug[:, :, j0:j0 + rows + 8, :]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for _ in range(3):
            sc.residual_ghosted(W)
        el = time.perf_counter() - t0
    return {'value': 3 * rows * NX / el, 'unit': UNIT, 'cores': 1, 'kind': 'oracle',
            'sample': '3 residual evaluations on a %dx%d-cell window (rows %d..%d) of the '
                      '1000x500 shock tube at t=0, numpy, 1 thread, %.1f s'
                      % (NX, rows, j0, j0 + rows - 1, el)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=100)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-rows', type=int, default=192)
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py measures one GPU only: this build has no multi-GPU path '
              '(the grid would be split into slabs with halo exchange; see the design notes).',
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_10569_amd import hweno, workloads

    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    U0 = torch.from_numpy(workloads.viscous_shock_tube_2d(NX, NY)).to(dev)
    s = hweno.Solver(NX, NY, extent=EXTENT, bc=BCS, device=dev, cfl=0.3, t_final=1.0, **PHYS)
    s.set_state(U0)
    for _ in range(args.warmup):
        s.rk_step(0.0)
    torch.cuda.synchronize()
    s.set_timing(True)
    s.timing(reset=True)
    restarts = 0
    pp = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d = s.rk_step(0.0)
        restarts += d['restarts']
        pp += d['pp_cells']
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = s.timing()
    _, t_end = s.get_state()

    cell_stages = args.steps * 3 * NX * NY
    value = cell_stages / el
    # dominant kernel by total GPU time
    dom = max(tm, key=lambda k: tm[k][0])
    ms, n = tm[dom]
    avg_s = ms / n / 1e3
    achieved = FLOPS[dom] * units_per_launch(dom) / avg_s / 1e12
    kern = {k: {'ms_total': round(v[0], 3), 'launches': v[1],
                'us_avg': round(1e3 * v[0] / v[1], 2) if v[1] else None}
            for k, v in tm.items()}
    path_flops = (FLOPS['recon'] + FLOPS['grad'] + FLOPS['rbar'] + FLOPS['update']
                  + 2 * FLOPS['flux'])
    out = {
        'metric': METRIC, 'value': value, 'unit': UNIT, 'n_gpus': 1,
        'steps': args.steps, 'warmup': args.warmup, 'ms_per_step': 1e3 * el / args.steps,
        'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64',
        'data': 'synthetic',
        'config': {'workload': '2D viscous shock tube 1000x500, Re=200, Pr=0.73, no-slip walls + '
                               'symmetry top, SSP-RK3 CFL 0.3 from t=0, paper dt rule',
                   'cells': NX * NY, 'stages_per_step': 3, 't_end': t_end,
                   'restarts': restarts, 'pp_cell_stages': pp},
        'roofline': {'bound': 'alu', 'kernel': dom, 'achieved': achieved,
                     'peak': PEAK_FP64_TFLOPS, 'unit': 'TFLOP/s',
                     'frac': achieved / PEAK_FP64_TFLOPS, 'traffic': None,
                     'flops_per_unit': FLOPS[dom], 'units_per_launch': units_per_launch(dom),
                     'us_per_launch': avg_s * 1e6},
        'hbm_frac_algorithmic': value * ALGO_BYTES_PER_CELL_STAGE / (PEAK_HBM_GBS * 1e9),
        'path_fp64_tflops_algorithmic': value * path_flops / 1e12,
        'kernels': kern,
    }
    if not args.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline(args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
