"""Why the inner operator keeps FP32 blocks (CPU, host-built blocks).

Iterative refinement x += S~^-1 (b - S x) with the exact inverse of an inner
operator S~ whose blocks are rounded: FP32 blocks reach the FP64 floor in
three steps, while blocks rounded to FP16 (with a power-of-two scale per
block, so they stay in range) or BF16 stall far above the 1e-10 target on
a structured cube, and on a 750-element jittered one FP16 blocks contract
slowly and BF16 blocks diverge (the contraction factor is about u kappa,
and kappa grows with the mesh).  Rounding every block
breaks S 1 = 0, so the rounded operator no longer shares the null space of
the anchored system and its low modes are wrong by about u kappa.
"""

import functools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from stdg_inputs import kuhn_mesh

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1601_07384_amd")


def assemble(B, cls, nbr, E, N, scale):
    rows, cols, vals = [], [], []
    for i in range(E):
        for k in range(5):
            t = i if k == 0 else nbr[i, k - 1]
            if t < 0:
                continue
            r, c = np.meshgrid(np.arange(N) + i * N, np.arange(N) + t * N, indexing="ij")
            rows.append(r.ravel()); cols.append(c.ravel()); vals.append(scale * B[cls[i], k].ravel())
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    keep = (rows != 0) & (cols != 0)                # pressure anchored at element 0, node 0
    rows = np.append(rows[keep], 0); cols = np.append(cols[keep], 0); vals = np.append(vals[keep], 1.0)
    return sp.csc_matrix((vals, (rows, cols)), shape=(E * N, E * N))


def rounded(B, kind):
    if kind == "fp32":
        return torch.tensor(B).float().double().numpy()
    if kind == "bf16":
        return torch.tensor(B).bfloat16().double().numpy()
    s = 2.0 ** np.ceil(np.log2(np.abs(B).max(axis=(2, 3), keepdims=True) + 1e-300))
    return torch.tensor(B / s).half().double().numpy() * s


@functools.lru_cache(maxsize=None)
def mesh_blocks(n, p, jitter):
    X, T = kuhn_mesh(n, jitter=jitter, seed=7)
    m = P.Mesh(X, T, p, 0, dt=1e-3, periodic=True, device=False)
    B, cls, nbr, C = m.blocks()
    return B, cls, nbr, C, m.E, m.N, assemble(B, cls, nbr, m.E, m.N, C[0, 0])


def refinement(n, p, jitter, kind, steps=10):
    B, cls, nbr, C, E, N, S = mesh_blocks(n, p, jitter)
    lu = spla.splu(assemble(rounded(B, kind), cls, nbr, E, N, C[0, 0]))
    rng = np.random.default_rng(0)
    xt = rng.standard_normal(S.shape[0])
    xt[0] = 0.0
    b = S @ xt
    x = np.zeros_like(b)
    hist = []
    for _ in range(steps):
        r = b - S @ x
        hist.append(np.linalg.norm(r) / np.linalg.norm(b))
        x = x + lu.solve(r)
    return hist


@pytest.mark.parametrize("n,p,jitter", [(4, 2, 0.0), (5, 3, 0.2)])
def test_fp32_blocks_refine_to_the_fp64_floor(n, p, jitter):
    h = refinement(n, p, jitter, "fp32")
    assert h[3] <= 1e-13


def test_16_bit_blocks_stall_on_a_structured_cube():
    for kind in ("fp16", "bf16"):
        h = refinement(4, 2, 0.0, kind)
        assert min(h) > 1e-10, (kind, h)


def test_16_bit_blocks_on_a_jittered_cube():
    """5^3 x 6 jittered tets, p = 3: FP16 blocks contract by about 0.2 per
    step and miss 1e-10 after ten steps, BF16 blocks diverge (on a 6^3 mesh
    FP16 diverges too: kappa grows with the mesh)."""
    h16 = refinement(5, 3, 0.2, "fp16")
    assert min(h16) > 1e-10, h16
    hb = refinement(5, 3, 0.2, "bf16")
    assert hb[-1] > hb[2] and min(hb) > 1e-10, hb
