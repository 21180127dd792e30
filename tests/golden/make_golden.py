"""Write the oracle's reference energies used by the GPU parity tests.

Calls only ``oracle/`` and the seeded input generators.  Run from the
repository root:  python tests/golden/make_golden.py
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dmrg as od  # noqa: E402
from oracle import fermions as fm  # noqa: E402
from oracle import submpo as sm  # noqa: E402
from workloads import WORKLOADS, chain_integrals, mps_values, workload_integrals  # noqa: E402

CASES = {
    # random molecule K=8, N=8, M=64, 6 sweeps
    "random_k8": dict(kind="workload", name="random_k8", M=64, sweeps=6),
    # the same molecule at M=256, where the two-site space is exact
    "random_k8_exact": dict(kind="workload", name="random_k8", M=256, sweeps=2),
    # chain K=8, N=8, M=16 (truncating), 3 sweeps
    "chain8": dict(kind="chain", K=8, N=8, seed=77, M=16, sweeps=3),
    # odd electron count: K=7, N=7, 2Sz=1
    "chain7_odd": dict(kind="chain", K=7, N=7, seed=78, M=16, sweeps=3),
    # chain8 on the compressed Hamiltonian (Sec. "Hamiltonian compression"):
    # threshold 0.037 lies in a gap of the singular values (0.0306, 0.0439)
    # and keeps 202 of 248 directions
    "chain8_compressed": dict(kind="chain", K=8, N=8, seed=77, M=16, sweeps=3, compress_tol=0.037),
    # chain8, chain7_odd and random_k8 on the stacked sub-Hamiltonian MPOs
    # (Sec. 4.2): grouping 0 = Eq. subH (first index), 1 = rightmost operator
    "chain8_subham0": dict(kind="chain", K=8, N=8, seed=77, M=16, sweeps=3, subham=0),
    "chain8_subham1": dict(kind="chain", K=8, N=8, seed=77, M=16, sweeps=3, subham=1),
    "chain7_odd_subham1": dict(kind="chain", K=7, N=7, seed=78, M=16, sweeps=3, subham=1),
    "random_k8_subham0": dict(kind="workload", name="random_k8", M=64, sweeps=6, subham=0),
}


def run(name, c):
    if c["kind"] == "workload":
        I = workload_integrals(c["name"])
        seed = WORKLOADS[c["name"]]["seed"]
    else:
        I = chain_integrals(c["K"], n_elec=c["N"], seed=c["seed"])
        seed = c["seed"]
    K, N, tsz, M = I.K, I.n_elec, I.two_sz, c["M"]
    n = od.n_mps_values(K, N, tsz, M)
    t0 = time.time()
    tol = c.get("compress_tol", 0.0)
    sub = c.get("subham")
    mpo = sm.build_sum_mpo(I.h, I.v, sub) if sub is not None else None
    d = od.DMRG(I.h, I.v, N, tsz, M, mps_values(seed, n), compress_tol=tol, mpo=mpo)
    sweeps = []
    for _ in range(c["sweeps"]):
        d.sweep()
        sweeps.append(d.log[-2]["theta"])
    thetas = [l["theta"] for l in d.log if "theta" in l][-2 * (K - 1):]
    out = dict(K=K, N=N, two_sz=tsz, M=M, seed=seed, kind=I.kind, sweeps=c["sweeps"],
               sweep_energies=sweeps, last_sweep_thetas=thetas, energy=d.energy(),
               bonds=[[list(q) + [dd] for q, dd in d.bond_sectors(k)] for k in range(K + 1)],
               compress_tol=tol, mpo_bond_dims=[len(ch) for ch in d.chans],
               subham=sub,
               seconds=time.time() - t0)
    if K <= 10:
        out["fci"] = fm.fci_energy(I.h, I.v, N, tsz)
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_dmrg.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for nm in names:
        data[nm] = run(nm, CASES[nm])
        data[nm]["source"] = "oracle/dmrg.py via tests/golden/make_golden.py"
        json.dump(data, open(path, "w"), indent=1)
        print(nm, data[nm]["energy"], "%.1fs" % data[nm]["seconds"], flush=True)
