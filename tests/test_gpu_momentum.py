"""Strategy-2 mean of the momentum 1-form (appendix C) on the GPU, through the C
ABI, against the oracle with the same option."""

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, compare_value, gpu_run, say

pytestmark = pytest.mark.gpu
MOM = ("S2_mom_x", "S2_mom_y")


def _oracle(w, steps, interp="bilinear", u=None, v=None, h=None):
    from oracle.lagmean import Params, Run
    if u is None:
        u, v, h = w.initial_state()
    r = Run(Params(N=w.N, dt=w.dt, f=w.f, g=w.g, H=w.H, nu8=w.nu8, interp=interp, momentum=True), u, v, h)
    r.begin_interval()
    r.step(steps)
    return r.end_interval()


def _gpu(w, steps, interp="bilinear", u=None, v=None, h=None):
    import paper_2208_02682_amd as lib
    if u is None:
        u, v, h = w.initial_state()
    run = lib.Run(lib.make_config(w.N, precision=w.precision, f=w.f, g=w.g, H=w.H, dt=w.dt, nu8=w.nu8,
                                  interp=interp, momentum=True))
    run.set_state(u, v, h)
    run.begin_interval()
    left = steps
    while left > 0:
        k = min(left, 256)
        run.step(k)
        left -= k
    run.end_interval()
    out = run.outputs()
    out.update(run.momentum_outputs())
    run.close()
    return out


def test_whole_64_interval_matches_the_oracle_and_leaves_the_rest_unchanged():
    from synth import workload
    w = workload("sw64_fp64")
    got = _gpu(w, w.steps_per_interval)
    ref = _oracle(w, w.steps_per_interval)
    for k in MOM + tuple(OUTPUT_KEYS):
        err = compare_value(k, got[k], ref[k])
        say(f"  {k}: rel {err:.3e}")
        assert err < 1e-12, (k, err)
    # the other outputs are bit for bit those of a run without the option
    run, plain = gpu_run(w, chunk=256)
    run.close()
    for k in OUTPUT_KEYS:
        assert np.array_equal(got[k], plain[0][k]), k


@pytest.mark.parametrize("N,prec,interp,steps,tol", [(128, "fp32", "bilinear", 150, 1e-5),
                                                     (192, "fp64", "cubic", 60, 1e-12),
                                                     (1024, "fp32", "bilinear", 3, 1e-5)])
def test_other_sizes_precisions_and_gathers(N, prec, interp, steps, tol):
    from synth.workloads import scaled_run
    w = scaled_run(N, Ro=0.08, ratio=1.0, periods=1.0, seeds=(71, 72), precision=prec)
    got = _gpu(w, steps, interp)
    ref = _oracle(w, steps, interp)
    for k in MOM:
        err = compare_value(k, got[k], ref[k])
        say(f"  N={N} {prec} {interp} {k}: rel {err:.3e}")
        assert err < tol, (k, err)


def test_steady_geostrophic_jet_gives_the_jet():
    from synth.workloads import Workload
    N = 64
    x = np.arange(N) * 2 * np.pi / N
    X, Y = np.meshgrid(x, x, indexing="xy")
    U = 0.2
    u, v, h = U * np.sin(Y), np.zeros((N, N)), 1.0 + U * np.cos(Y)
    w = Workload(name="jet", N=N, precision="fp64", k0=1.0, Ro=0.1, k_lo=1.0, k_hi=1.0, ratio=1.0,
                 seed_vortex=0, seed_wave=0, dt=0.05, steps_per_interval=60, n_intervals=1, nu8=0.0)
    got = _gpu(w, 60, u=u, v=v, h=h)
    assert np.max(np.abs(got["S2_mom_x"] - u)) < 1e-12 and np.max(np.abs(got["S2_mom_y"])) < 1e-12


def test_momentum_runs_batched_are_the_same_as_alone():
    import paper_2208_02682_amd as lib
    from synth.workloads import scaled_run
    specs = [(64, "fp64", True, 21), (64, "fp64", False, 13), (128, "fp32", True, 17)]
    ws = [scaled_run(N, Ro=0.06, ratio=1.1, periods=1.0, seeds=(80 + 2 * i, 81 + 2 * i), precision=p)
          for i, (N, p, _, _) in enumerate(specs)]

    def start(w, mom):
        r = lib.Run(lib.make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8, momentum=mom))
        r.set_state(*w.initial_state())
        r.begin_interval()
        return r

    def outs(r, mom):
        o = r.outputs()
        if mom:
            o.update(r.momentum_outputs())
        return o

    alone = []
    for w, (_, _, mom, steps) in zip(ws, specs):
        r = start(w, mom)
        r.step(steps)
        r.end_interval()
        alone.append(outs(r, mom))
        r.close()
    runs = [start(w, sp[2]) for w, sp in zip(ws, specs)]
    with lib.Batch() as b:
        for r, sp in zip(runs, specs):
            b.add(r, sp[3])
        while b.step(6):
            pass
        for r in runs:
            b.remove(r)
    for i, (r, sp) in enumerate(zip(runs, specs)):
        r.end_interval()
        got = outs(r, sp[2])
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (i, k)
        r.close()


def test_reading_the_momentum_of_a_run_without_it_is_refused():
    import paper_2208_02682_amd as lib
    from paper_2208_02682_amd import LagMeanError
    from synth import workload
    w = workload("sw64_fp64")
    run, _ = gpu_run(w, steps_per_interval=3, n_intervals=1)
    with pytest.raises(LagMeanError) as e:
        run.momentum_outputs()
    assert e.value.status == -2
    run.close()
