"""Batched execution: many 2D grids of different sizes and physics in one
graph launch.  Every instance must come out bitwise identical to the same
problem advanced alone by the single-grid path (which the other GPU tests tie
to the oracle), whatever the tiles and instance order; restarts, bad inputs
and t_final are per instance."""

import numpy as np
import pytest

torch = pytest.importorskip('torch')

from paper_2608_10569_amd import hweno, workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = 'cuda:0'


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(DEV)


def single_run(prob, U, nsteps):
    kw = dict(prob)
    nx, ny = kw.pop('nx'), kw.pop('ny')
    s = hweno.Solver(nx, ny, **kw)
    s.set_state(to_dev(U))
    steps, restarts = 0, 0
    for _ in range(nsteps):
        d = s.rk_step(0.0)
        if d['dt'] == 0.0:
            break
        steps += 1
        restarts += d['restarts']
    U1, t = s.get_state()
    return U1, t, steps, restarts


def mixed_problems():
    probs, states = [], []
    specs = [(16, 12, 0.01, ('periodic',) * 4, (0.0, 1.0, 0.0, 1.0)),
             (24, 24, 1e-3, ('periodic',) * 4, (0.0, 1.0, 0.0, 1.0)),
             (32, 16, 5e-3, ('noslip', 'noslip', 'noslip', 'slip'), (0.0, 1.0, 0.0, 0.5)),
             (12, 20, 2e-2, ('periodic',) * 4, (0.0, 1.0, 0.0, 1.0)),
             (40, 36, 1e-4, ('outflow', 'slip', 'slip', 'outflow'), (0.0, 1.0, 0.0, 1.0))]
    for k, (nx, ny, mu, bc, ext) in enumerate(specs):
        probs.append(dict(nx=nx, ny=ny, mu_ref=mu, bc=bc, extent=ext))
        states.append(workloads.random_smooth_2d(nx, ny, seed=40 + k, noise=1e-3, extent=ext))
    return probs, states


def run_batch(probs, states, nsteps, tiles=None):
    b = hweno.Batch(probs)
    if tiles:
        b.set_tiles(**tiles)
    for i, U in enumerate(states):
        b.set_state(i, to_dev(U))
    b.run(nsteps)
    return b


def test_batch_equals_single_grids():
    probs, states = mixed_problems()
    nsteps = 6
    b = run_batch(probs, states, nsteps)
    for i, (p, U) in enumerate(zip(probs, states)):
        ref, t, steps, _ = single_run(p, U, nsteps)
        got, tb = b.get_state(i)
        d = b.diag(i)
        print('instance %d %dx%d: t %.6e vs %.6e, steps %d, equal %s'
              % (i, p['nx'], p['ny'], tb, t, d['steps'], torch.equal(got, ref)))
        assert d['steps'] == nsteps and tb == t
        assert torch.equal(got, ref)


def test_batch_mixed_viscosity_laws_equal_single_grids():
    """One instance with mu(T) makes the whole launch use the kernels built
    with the power law; the constant-viscosity instances beside it must still
    match their single-grid runs (which use the constant-viscosity build)
    bit for bit, with the face fluxes split and fused."""
    probs, states = mixed_problems()
    probs = probs[:3]
    states = states[:3]
    probs[1] = dict(probs[1], mu_exp=0.7, T_ref=1.0 / 1.4)
    for tiles in (dict(recon=32, grad=64, flux=0, order=0, xcd=1),
                  dict(recon=32, grad=32, flux=64, order=0, xcd=1),
                  dict(recon=32, grad=0, flux=0, order=0, xcd=1)):
        b = run_batch(probs, states, 4, tiles)
        for i, (p, U) in enumerate(zip(probs, states)):
            ref, t, steps, _ = single_run(p, U, 4)
            got, tb = b.get_state(i)
            print('flux %d, instance %d (mu_exp %s): equal %s'
                  % (tiles['flux'], i, p.get('mu_exp', 0.0), torch.equal(got, ref)), flush=True)
            assert tb == t and torch.equal(got, ref)


@pytest.mark.parametrize('tiles', [dict(recon=16, grad=64, flux=128, order=1, xcd=1),
                                   dict(recon=32, grad=32, flux=64, order=1, xcd=0),
                                   dict(recon=16, grad=32, flux=128, order=0, xcd=0),
                                   dict(recon=32, grad=64, flux=0, order=1, xcd=1),
                                   dict(recon=16, grad=0, flux=0, order=1, xcd=1),
                                   dict(recon=32, grad=0, flux=64, order=0, xcd=0)])
def test_batch_tiles_do_not_change_results(tiles):
    probs, states = mixed_problems()
    a = run_batch(probs, states, 3)
    b = run_batch(probs, states, 3, tiles)
    assert b.tiles() == tiles
    for i in range(len(probs)):
        assert torch.equal(a.get_state(i)[0], b.get_state(i)[0])


def test_single_grid_tiles_and_autotune():
    U = workloads.random_smooth_2d(30, 22, seed=50, noise=1e-3)
    ref = hweno.Solver(30, 22, mu_ref=0.01)
    ref.set_state(to_dev(U))
    for _ in range(3):
        ref.rk_step(0.0)
    s = hweno.Solver(30, 22, mu_ref=0.01)
    s.set_state(to_dev(U))
    chosen = s.autotune(reps=2)
    assert chosen['recon'] in (16, 32) and chosen['grad'] in (0, 32, 64)
    assert chosen['flux'] in (0, 64, 128)
    assert chosen['xcd'] in (0, 1)
    assert torch.equal(s.get_state()[0], to_dev(U))          # the tuner leaves the state alone
    for _ in range(3):
        s.rk_step(0.0)
    assert torch.equal(s.get_state()[0], ref.get_state()[0])


def test_batch_autotune_keeps_results():
    probs, states = mixed_problems()
    a = run_batch(probs, states, 2)
    b = hweno.Batch(probs)
    for i, U in enumerate(states):
        b.set_state(i, to_dev(U))
    chosen = b.autotune(reps=2)
    print('batch autotune:', chosen)
    b.run(2)
    for i in range(len(probs)):
        assert torch.equal(a.get_state(i)[0], b.get_state(i)[0])


def trough_state(n=16):
    U = workloads.random_smooth_2d(n, n, seed=7, noise=1e-3)
    U[0, 0, 6:9, 5:10] = 2e-3
    U[0, 3, 6:9, 5:10] = 0.5 * (U[0, 1, 6:9, 5:10] ** 2 + U[0, 2, 6:9, 5:10] ** 2) / 2e-3 + 2e-3
    U[1:, :, 6:9, 5:10] = 0.0
    return U


def test_batch_restarts_per_instance():
    """An instance whose rule step is inadmissible restarts with dt/2 on its
    own; the others are unaffected and every instance matches its single run."""
    U = trough_state()
    restart_prob = None
    for cfl in (1.0, 2.0, 4.0, 8.0):
        p = dict(nx=16, ny=16, mu_ref=0.01, cfl=cfl)
        try:
            _, _, steps, restarts = single_run(p, U, 2)
        except hweno.HwenoError:
            continue
        if restarts > 0:
            restart_prob = p
            break
    assert restart_prob is not None, 'no CFL in the list makes the trough state restart'
    probs, states = mixed_problems()
    probs = probs[:2] + [restart_prob] + probs[2:]
    states = states[:2] + [U] + states[2:]
    nsteps = 2
    b = run_batch(probs, states, nsteps)
    for i, (p, S) in enumerate(zip(probs, states)):
        ref, t, steps, restarts = single_run(p, S, nsteps)
        got, tb = b.get_state(i)
        d = b.diag(i)
        print('instance %d: restarts %d (single %d), steps %d, t %.6e vs %.6e'
              % (i, d['restarts'], restarts, d['steps'], tb, t))
        assert d['restarts'] == restarts and d['steps'] == steps == nsteps and tb == t
        assert torch.equal(got, ref)
    assert b.diag(2)['restarts'] > 0


def test_batch_bad_input_and_t_final():
    probs, states = mixed_problems()
    bad = states[1].copy()
    bad[0, 0, 3, 4] = -1.0
    states = [states[0], bad, states[2]]
    probs = [probs[0], probs[1], dict(probs[2], t_final=1e-3)]
    b = hweno.Batch(probs)
    for i, U in enumerate(states):
        b.set_state(i, to_dev(U))
    with pytest.raises(hweno.HwenoError) as e:
        b.run(50)
    assert e.value.code == 5
    # the bad instance did not move; the others ran
    assert torch.equal(b.get_state(1)[0], to_dev(bad))
    ref, t, steps, _ = single_run(probs[0], states[0], 50)
    assert torch.equal(b.get_state(0)[0], ref) and b.diag(0)['steps'] == 50
    # t_final: stops exactly there, fewer steps
    ref2, t2, steps2, _ = single_run(probs[2], states[2], 50)
    d2 = b.diag(2)
    assert d2['steps'] == steps2 < 50 and d2['t'] == t2 and abs(t2 - 1e-3) < 1e-15
    assert torch.equal(b.get_state(2)[0], ref2)


def test_c4_batch_sampled_instances():
    """The 64-instance workload (grids 64^2..512^2, Re 1e2..1e4): two steps in
    one graph; the smallest, the largest and one more instance against their
    single-grid runs."""
    inst = workloads.batched_periodic_2d()
    probs = [dict(nx=n, ny=n, mu_ref=1.0 / Re) for n, Re, _ in inst]
    b = hweno.Batch(probs)
    for i, (_, _, U) in enumerate(inst):
        b.set_state(i, to_dev(U))
    b.run(2)
    sizes = [n for n, _, _ in inst]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17})
    for i in picks:
        ref, t, _, _ = single_run(probs[i], inst[i][2], 2)
        got, tb = b.get_state(i)
        print('C4 instance %d (%d^2, Re %.0f): equal %s' % (i, sizes[i], inst[i][1], torch.equal(got, ref)))
        assert tb == t and torch.equal(got, ref)


def test_full_batch_two_chains_equal_single_grids():
    """The benchmark's 64-instance batch (two concurrent chains in its graph)
    over 50 steps: one instance of each size, and the last instance of each
    chain, equal the same problems advanced alone, bit for bit."""
    inst = workloads.batched_periodic_2d()
    probs = [dict(nx=n, ny=n, mu_ref=1.0 / Re) for n, Re, _ in inst]
    b = hweno.Batch(probs)
    for i, (_, _, U) in enumerate(inst):
        b.set_state(i, to_dev(U))
    b.run(50)
    picks = {}
    for i, (n, _, _) in enumerate(inst):
        picks.setdefault(n, i)
    for i in sorted(set(picks.values()) | {len(inst) // 2 - 1, len(inst) - 1}):
        ref, t, steps, _ = single_run(probs[i], inst[i][2], 50)
        got, tb = b.get_state(i)
        print('instance %d (%d^2): t %.6e vs %.6e, equal %s'
              % (i, inst[i][0], tb, t, torch.equal(got, ref)), flush=True)
        assert b.diag(i)['steps'] == 50 and tb == t and torch.equal(got, ref)
