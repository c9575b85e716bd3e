"""Generator invariants: the known optimum is primal/dual feasible and
complementary, so it satisfies the KKT conditions of Sec. 2.2 exactly."""
import numpy as np
import pytest

from paper_2412_07731_amd import gen


@pytest.mark.parametrize("seed", range(4))
def test_known_optimum_kkt(seed):
    inst = gen.generate("tiny", seed)
    xs, ys, zs = inst.xstar, inst.ystar, inst.zstar
    # independent dense operator built from the blocks
    A = dense_operator(inst)
    assert np.allclose(A @ xs, inst.b, rtol=0, atol=1e-13)
    assert np.allclose(A.T @ ys + zs, inst.c, rtol=0, atol=1e-13)
    assert np.all(xs >= 0) and np.all(zs >= 0)
    assert np.all(xs * zs == 0)
    assert abs(inst.c @ xs - inst.b @ ys) <= 1e-12 * (1 + abs(inst.fstar))


def dense_operator(inst):
    """Write the constraint matrix out entry block by entry block."""
    xo, yo, lo = inst.xoff(), inst.yoff(), inst.loff()
    A = np.zeros((inst.m_tot, inst.n_tot))
    for i in range(inst.N):
        A[yo[i]:yo[i + 1], xo[i]:xo[i + 1]] = inst.A[i]
        A[yo[i]:yo[i + 1], xo[-1]:] = inst.C[i]
    for j in range(inst.N - 1):
        r = slice(yo[-1] + lo[j], yo[-1] + lo[j + 1])
        A[r, xo[j]:xo[j + 1]] = inst.FR[j]
        A[r, xo[j + 1]:xo[j + 2]] = inst.FL[j]
    return A


def test_shapes_and_structure():
    inst = gen.generate("tiny", 3)
    assert inst.N == 8 and inst.n0 == 8
    assert inst.n_tot == 8 * 64 + 8 and inst.m_tot == 8 * 32 + 7 * 4
    for j in range(inst.N - 1):
        # storage continuity: +1 on the last l variables of block j,
        # -1 on the first l variables of block j+1
        assert np.array_equal(inst.FR[j][:, -4:], np.eye(4))
        assert np.array_equal(inst.FL[j][:, :4], -np.eye(4))
        assert np.count_nonzero(inst.FR[j]) == 4 and np.count_nonzero(inst.FL[j]) == 4
    for i in range(inst.N):
        assert np.all(np.any(inst.A[i] != 0, axis=1)), "no all-zero rows"
        assert np.linalg.matrix_rank(inst.A[i]) == inst.m[i]
        xi = inst.xstar[inst.xoff()[i]:inst.xoff()[i + 1]]
        assert np.count_nonzero(xi) == inst.n[i] // 2
    dens = np.mean([np.count_nonzero(a) / a.size for a in inst.A])
    assert 0.25 < dens < 0.35


def test_basis_unique_primal():
    """x* is the unique primal optimum: the columns of its support have full
    column rank."""
    inst = gen.generate("tiny", 1)
    A = dense_operator(inst)
    B = np.flatnonzero(inst.xstar > 0)
    assert np.linalg.matrix_rank(A[:, B]) == B.size


def test_uneven_sizes_and_determinism():
    cfg = dict(gen.CONFIGS["uneven"], N=6)
    a = gen.generate(cfg, 5)
    b = gen.generate(cfg, 5)
    assert np.array_equal(a.m, b.m) and np.array_equal(a.l, b.l)
    assert all(np.array_equal(x, y) for x, y in zip(a.A, b.A))
    assert np.all((a.m >= 64) & (a.m <= 512)) and np.array_equal(a.n, 2 * a.m)
    assert np.all((a.l >= 4) & (a.l <= 32))
    c = gen.generate(cfg, 6)
    assert not np.array_equal(a.b[:10], c.b[:10])


def test_nondegenerate_variant_has_square_nonsingular_basis():
    """tiny_nd: exactly m_tot positive x* entries, the basis matrix square and
    nonsingular, strict complementarity, and the first l_{i-1} variables of
    every block outside the basis (A_B block diagonal)."""
    import numpy as np
    from oracle import lp
    inst = gen.generate("tiny_nd", 0)
    assert inst.n0 == 0 and inst.basis is not None
    xo, _, _ = lp.offsets(inst)
    cols = np.concatenate([xo[i] + inst.basis[i] for i in range(inst.N)])
    assert cols.size == inst.m_tot == int(np.count_nonzero(inst.xstar))
    AB = lp.full_matrix(inst).toarray()[:, cols]
    assert np.linalg.matrix_rank(AB) == inst.m_tot
    assert np.all((inst.xstar > 0) != (inst.zstar > 0))
    for i in range(1, inst.N):
        assert np.all(inst.basis[i] >= inst.l[i - 1])
    assert abs(inst.c @ inst.xstar - inst.b @ inst.ystar) <= 1e-9 * abs(inst.fstar)
