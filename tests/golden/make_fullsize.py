"""Writes fullsize_<workload>.json: oracle values for the full-size parity
test of the benchmark workload, which the oracle cannot recompute inside a
GPU test in seconds.

Calls only oracle/ and the seeded input generator:
  * sha256 of the oracle CSR row pointers and column indices, and the ground
    node (the HIP structure must match bit for bit);
  * 2000 sampled CSR values (positions seeded);
  * oracle PCG iteration counts (Jacobi, tol 1e-8) for 2 electrode columns;
  * 6 lead-field columns by reciprocity (oracle PCG at tol 1e-12 on the
    Schur system).

    python tests/golden/make_fullsize.py [workload]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem, leadfield as lf, solve, source  # noqa: E402
from paper_1811_07717_amd import headmodel as hm  # noqa: E402

LF_COLUMNS = [0, 3 * 1234 + 1, 3 * 5000 + 2, 3 * 7777, 3 * 9000 + 1, 29999]
# the 1 mm workload has 100 000 dipoles: columns spread over all of them
LF_COLUMNS_1MM = [0, 3 * 1234 + 1, 3 * 31415 + 2, 3 * 50000, 3 * 77777 + 1, 299999]
PCG_COLUMNS = [0, 77]


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(name="sphere2mm_L128"):
    t0 = time.time()
    H = hm.workload(name)
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    A = S["A"]
    print("assembled", time.time() - t0, flush=True)
    rng = np.random.default_rng(2024)
    pos = np.sort(rng.choice(A.nnz, size=2000, replace=False))
    d = fem.preconditioner_diag(A)
    its = {}
    for c in PCG_COLUMNS:
        _, k, _ = solve.pcg(A, S["B"][:, [c]].toarray().ravel(), d, tol=1e-8)
        its[str(c)] = int(k)
        print("pcg column", c, k, time.time() - t0, flush=True)
    G = source.point_dipole_matrix(H.nodes, H.tets, H.dipole_tets)
    wanted = LF_COLUMNS_1MM if G.shape[1] >= 300000 else LF_COLUMNS
    cols = [c for c in wanted if c < G.shape[1]]
    LFc = lf.leadfield_columns_reciprocity(A, S["B"], S["C"], G[:, cols], tol=1e-12)
    print("lead-field columns", time.time() - t0, flush=True)
    out = {
        "_source": "tests/golden/make_fullsize.py (oracle only)",
        "workload": name, "n": H.n, "e": H.e, "L": H.L, "nnz": int(A.nnz),
        "ground": int(S["ground"]),
        "row_ptr_sha256": sha(A.indptr.astype(np.int32)),
        "col_sha256": sha(A.indices.astype(np.int32)),
        "sample_pos": pos.tolist(), "sample_val": A.data[pos].tolist(),
        "pcg_iters": its,
        "lf_columns": cols, "lf_values": LFc.T.tolist(),
    }
    with open(os.path.join(HERE, f"fullsize_{name}.json"), "w") as f:
        json.dump(out, f)
    print("written", time.time() - t0)


if __name__ == "__main__":
    main(*sys.argv[1:])
