"""Write oracle reference values for the large workloads (c3, c4, c5).

Calls only the CPU oracle and the seeded input generators; the GPU tests
regenerate the same inputs (checked by SHA-256) and compare against these
values.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import oracle_ewald  # noqa: E402
from paper_2408_03273_amd import workloads as wl  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def sample_idx(n, k, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=min(k, n), replace=False))
    # always include the first and last rows (tile edges)
    return np.unique(np.concatenate([[0, n - 1], idx])).astype(int)


def ref(sys_, mm_sel):
    r = oracle_ewald(sys_.box, sys_.alpha, sys_.rcut, sys_.kmax, sys_.qm_pos, sys_.Q, sys_.mu, sys_.theta,
                     sys_.mm_pos, sys_.q, mm_sel=mm_sel)
    return dict(energy=r.E, phi=r.phi.tolist(), efield=(-r.dphi).tolist(), efgrad=(-2 * r.hphi).tolist(),
                g_qm_pos=r.g_qm_pos.tolist(), g_Q=r.g_Q.tolist(), g_mu=r.g_mu.tolist(), g_theta=r.g_theta.tolist(),
                mm_sel=[int(i) for i in mm_sel], g_mm_pos=r.g_mm_pos.tolist(), g_mm_q=r.g_mm_q.tolist())


def main():
    # c3 and the first c4 frames with larger MM samples; every other c4 frame
    # (each has its own size, box and packed offset in the batch) and the
    # middle and last c5 replicas with smaller ones
    jobs = [("c3_f0", 3, 0, 1500), ("c4_f0", 4, 0, 600), ("c4_f1", 4, 1, 600), ("c4_f2", 4, 2, 600),
            ("c5_f0", 5, 0, 400)]
    jobs += [(f"c4_f{f}", 4, f, 200) for f in range(3, 64)]
    jobs += [("c5_f7", 5, 7, 200), ("c5_f15", 5, 15, 200)]
    only = sys.argv[1:]
    for name, cfg, frame, nsel in jobs:
        if only and name not in only:
            continue
        s = wl.make_config(cfg, frame)
        sel = sample_idx(s.nm, nsel, 1000 * cfg + frame)
        t = time.time()
        d = ref(s, sel)
        d.update(name=name, config=cfg, frame=frame, input_sha256=s.sha256(), nq=s.nq, nm=s.nm,
                 oracle_seconds=round(time.time() - t, 1))
        with open(os.path.join(OUT, f"oracle_{name}.json"), "w") as f:
            json.dump(d, f)
        print(name, s.nq, s.nm, f"{time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main()
