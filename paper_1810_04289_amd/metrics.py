"""Algorithmic byte counts of the hot kernels, for rooflines: what each launch must move
through HBM at least, from the solver's sizes and Schwarz pattern."""
from __future__ import annotations

import numpy as np


def sweep_bytes(s, precision: int = 0) -> dict:
    """Algorithmic HBM bytes of one launch of each triangular sweep of the Schwarz solve,
    with factor entries of vb bytes (8 FP64, 4 FP32, 2 BF16) and local values of yb bytes
    (8 FP64, else 4).

    forward  (y = L^-1 R v): strict-L blocks (49 vb each) and their column slot (4 B), a
             24 B task record per local row, the gathered FP64 input (7 doubles per local
             row) and y written (7 yb per local row);
    backward (x = U^-1 y): strict-U blocks and the inverted diagonal of every row (49 vb
             each), the U column slots, the task records, y read, and the owned rows of z
             written (7 doubles per vertex).
    """
    vb = {0: 8, 1: 4, 2: 2, 3: 4}[precision]
    yb = 8 if precision == 0 else 4
    pc = s.pc_get(factors=False)
    ns = len(pc["sub_nowned"])
    rp = pc["lrowptr"].astype(np.int64)
    col = pc["lcolind"].astype(np.int64)
    nL = 0
    for k in range(ns):
        r0 = int(pc["sub_ptr"][k]) + k          # row pointers of subdomain k start here
        n_k = int(pc["sub_ptr"][k + 1] - pc["sub_ptr"][k])
        ptr = rp[r0:r0 + n_k + 1]
        b0 = int(pc["blk_ptr"][k])
        rows = np.repeat(np.arange(n_k), np.diff(ptr))
        nL += int(np.count_nonzero(col[b0 + ptr[0]:b0 + ptr[-1]] < rows))
    NB = len(col)
    R = len(pc["sub_verts"])
    nU = NB - R - nL
    fwd = nL * (49 * vb + 4) + 24 * R + 56 * R + 7 * yb * R
    bwd = (nU + R) * 49 * vb + 4 * nU + 24 * R + 7 * yb * R + 56 * s.V
    return dict(ilu_fwd=fwd, ilu_bwd=bwd, local_blocks=NB, local_rows=R, l_blocks=nL, u_blocks=nU)


def spmv_bytes(s) -> int:
    """Algorithmic bytes of y = J x: blocks once, column indices, row pointers, x and y once."""
    return s.nnzb * (49 * 8 + 4) + 4 * (s.V + 1) + 2 * 7 * s.V * 8
