"""Write the Lanczos-oracle eigenvalues of the single-vector workload's field
distribution (T x L^3 random SU(3) x U(1), eps 0.2, seed 1, charge -1/3,
kappa 0.1365, c_sw 1.9 / 1.0): the 8 eigenvalues of Q smallest in modulus,
one per Kramers pair (sign-of-the-Pfaffian section: the spectrum of Q is
doubly degenerate), with their rigorous residual bounds.

Calls only the oracle (oracle.lanczos over oracle.dirac) and the seeded input
generator.  Usage (repository root):

    python tests/golden/make_lanczos_golden.py 8      # 8x8^3, minutes
    python tests/golden/make_lanczos_golden.py 16     # 16x16^3 (the workload's size), about an hour on 8 cores
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dirac, lanczos  # noqa: E402
from paper_2108_11989_amd import synth  # noqa: E402

K, GUARD, DEGREE, TOL = 8, 2, 12, 1e-13
EPS, SEED, Q, KAPPA = 0.2, 1, -1.0 / 3.0, 0.1365


def main(L: int):
    T = L
    su3, th = synth.make_field(T, L, EPS, SEED)
    op = dirac.Operator(su3, th, Q, synth.CSW_SU3, synth.CSW_U1)
    m0 = float(synth.kappa_to_m0(KAPPA))
    t0 = time.time()
    ev, err, applies = lanczos.lowest_q(op, m0, K, guard=GUARD, tol=TOL, degree=DEGREE,
                                        log=lambda s: print(s, flush=True))
    out = {
        "what": "8 eigenvalues of Q(m0) smallest in modulus, one per Kramers pair, signed, sorted by |lambda|; "
                "err: residual norm ||Q z - lambda z|| of each unit Ritz vector (a rigorous bound)",
        "source": "oracle.lanczos.lowest_q (FP64 thick-restart Lanczos on a Chebyshev polynomial of Q^2, "
                  "Rayleigh-Ritz with Q on the Kramers-closed span); written by tests/golden/make_lanczos_golden.py",
        "lattice": [T, L], "eps": EPS, "seed": SEED, "q": Q, "kappa": KAPPA, "m0": m0,
        "csw_su3": synth.CSW_SU3, "csw_u1": synth.CSW_U1, "time_bc": 1,
        "k": K, "guard": GUARD, "degree": DEGREE, "tol": TOL,
        "evals": [float(x) for x in ev], "err": [float(x) for x in err],
        "q_applies": int(applies), "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"c1_lanczos_{T}x{L}x{L}x{L}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["evals"], out["err"], flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]))
