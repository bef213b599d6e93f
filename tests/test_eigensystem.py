"""Host logic of the split-BF16 path: the eigen-decomposition from which its
transition matrices are formed, exp(Q tau) - I = V (exp(B tau) - I) V^-1,
checked against scipy's expm (a different method: Pade scaling and
squaring) and against the defining relations Q V = V B, V V^-1 = I.  No GPU.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1905_12146_amd import binding as B
from synth.workloads import codon_rate_matrix, random_rate_matrix
from tests._fixtures import jc_matrix


def block_b(re, im, kind):
    m = len(re)
    Bm = np.zeros((m, m))
    for j in range(m):
        if kind[j] == 0:
            Bm[j, j] = re[j]
        elif kind[j] == 1:
            Bm[j, j] = Bm[j + 1, j + 1] = re[j]
            Bm[j, j + 1] = im[j]
            Bm[j + 1, j] = -im[j]
    return Bm


def f_of(V, Vinv, re, im, kind, tau):
    """V (exp(B tau) - I) V^-1, the blocks written out as the kernels do."""
    m = len(re)
    E = np.zeros((m, m))
    for j in range(m):
        if kind[j] == 0:
            E[j, j] = np.expm1(re[j] * tau)
        elif kind[j] == 1:
            a, b = re[j] * tau, im[j] * tau
            c = np.expm1(a) * np.cos(b) - 2 * np.sin(b / 2) ** 2
            s = np.exp(a) * np.sin(b)
            E[j, j] = E[j + 1, j + 1] = c
            E[j, j + 1] = s
            E[j + 1, j] = -s
    return V @ E @ Vinv


def rate_matrices():
    rng = np.random.default_rng(2024)
    out = [("random%d" % m, random_rate_matrix(m, rng)) for m in (2, 3, 4, 20, 61, 64)]
    out.append(("codon", codon_rate_matrix(rng.dirichlet(np.ones(61)), np.exp(1.0), np.exp(-1.0), rng)))
    cyc = np.zeros((5, 5))
    for x in range(5):
        cyc[x, (x + 1) % 5] = 1.0
        cyc[x, (x + 2) % 5] = 0.1
    np.fill_diagonal(cyc, -cyc.sum(axis=1))
    out.append(("cyclic", cyc))   # complex pairs
    out.append(("jc", jc_matrix(4)))  # a triple eigenvalue
    return out


def _q(case):
    Q = case[1]
    return Q[0] if isinstance(Q, tuple) else Q


@pytest.mark.parametrize("case", rate_matrices(), ids=lambda c: c[0])
def test_decomposition_reconstructs_q(case):
    Q = _q(case)
    V, Vinv, re, im, kind, cond, resid = B.pg_eigensystem(Q)
    scale = np.abs(Q).max()
    assert resid <= 1e-11 and cond <= 1e6, (resid, cond)
    assert np.abs(V @ block_b(re, im, kind) @ Vinv - Q).max() <= 1e-11 * scale
    assert np.abs(Q @ V - V @ block_b(re, im, kind)).max() <= 1e-11 * scale * np.abs(V).max()
    assert np.abs(V @ Vinv - np.eye(len(Q))).max() <= 1e-11 * cond


@pytest.mark.parametrize("case", rate_matrices(), ids=lambda c: c[0])
def test_transition_matrices_match_expm(case):
    Q = _q(case)
    V, Vinv, re, im, kind, cond, resid = B.pg_eigensystem(Q)
    for tau in (1e-5, 1e-2, 0.3, 3.0):
        F = f_of(V, Vinv, re, im, kind, tau)
        ref = sl.expm(Q * tau) - np.eye(len(Q))
        assert np.abs(F - ref).max() <= 1e-11 * max(np.abs(ref).max(), 1e-300), (tau,)


def test_complex_pairs_found():
    Q = _q(rate_matrices()[-2])
    _, _, re, im, kind, _, _ = B.pg_eigensystem(Q)
    assert (kind == 1).sum() == 2 and (kind == 2).sum() == 2
    lam = np.linalg.eigvals(Q)
    got = np.concatenate([re[kind == 0], re[kind == 1] + 1j * im[kind == 1], re[kind == 1] - 1j * im[kind == 1]])
    assert np.abs(np.sort_complex(got) - np.sort_complex(lam)).max() <= 1e-12


def test_non_diagonalisable_is_flagged():
    Q = np.array([[-1.0, 1.0, 0.0], [0.0, -1.0, 1.0], [0.0, 0.0, 0.0]])
    try:
        _, _, _, _, _, cond, resid = B.pg_eigensystem(Q)
    except B.PhyloGradError as e:
        assert e.code == B.PG_E_MODEL
        return
    assert resid > 1e-11 or cond > 1e6


def test_split_footprint():
    fp = B.pg_footprint_bytes(256, 1000, 61, 4, B.PG_SPLIT_BF16)
    vec = 4 * 64 * 1008 * 255 * 4
    assert 2 * vec + 49152 * 510 * 4 <= fp <= 2 * vec + 49152 * 510 * 4 + 16 * 2**20
