"""Host-side logic of bench.py (no GPU): the one-GPU refusal, and the
closure row's comparison with the FP64 oracle's own fine run."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    for extra, env in [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})]:
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + extra,
                           capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, **env))
        assert r.returncode == 2, r.stderr
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_closure_vs_oracle_measures_against_the_oracle_fine_run():
    """closure_vs_oracle runs the oracle on the case for warmup + 2k steps and
    restricts it: the oracle's own restricted state scores 0, a state off by
    1 % everywhere scores 0.01, and a state shifted by a constant scores its
    norm ratio."""
    import bench
    import oracle
    from oracle import closure as oc
    from paper_1305_3976_amd import inputs

    nf, warm, k = 16, 2, 1
    case = inputs.closure_family(1, seed=3, n_fine=nf)[0]
    P = oracle.make_params(3, (nf, nf, nf), 1.0 / nf, rho=1.0, mu=0.01, dt=case.dt_fine)
    S = case.structure
    sim = oracle.Sim(P, [np.asarray(c, dtype=np.float64) for c in case.u0], S.X, S.links, S.w)
    sim.advance(warm + 2 * k)
    ref = [oc.restrict_face(sim.u[c], c) for c in range(3)]
    assert ref[0].shape == (nf // 2,) * 3
    shift = [r + 1e-3 for r in ref]
    keep = {"case": case, "n_fine": nf, "warmup": warm,
            "snap": {"interval": k, "fine": ref, "plain": [1.01 * r for r in ref],
                     "corrected": shift}}
    out = bench.closure_vs_oracle(keep)
    e = out["rel_l2_vs_restricted_oracle"]
    assert out["oracle_fine_steps"] == warm + 2 * k
    assert e["gpu_fine_restricted"] == 0.0
    assert abs(e["plain_coarse"] - 0.01) < 1e-6
    want = 1e-3 * np.sqrt(3 * (nf // 2) ** 3) / np.sqrt(sum(float(np.sum(r ** 2)) for r in ref))
    assert abs(e["coarse_plus_closure"] - want) <= 1e-6 * max(1.0, want)
