"""The allocation-free local product (tt_local_matvec_noalloc) through the C ABI
against tt_local_matvec on the same inputs: two calls in a row, the second with
a smaller system (its scratch starts with the first call's contents), FP64 and
the mixed-precision products, plus the size limit and the oracle's dense
projected operator for the FP64 result."""
import numpy as np
import pytest
import torch

from oracle import tt as ott

pytestmark = pytest.mark.gpu


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _system(P, rng, r, rp, R, R2, m=4, precision=0):
    """Two components; a single block, an identity block and a chain of two
    projected operators (the reduced system's L_X^ Aeq^T^ pattern)."""
    def op(Ra, Rb):
        return (rng.standard_normal((r, Ra, r)), rng.standard_normal((Ra, m, m, Rb)),
                rng.standard_normal((rp, Rb, rp)))
    o1, o2, o3 = op(R, R2), op(R2, R), op(R, R)
    ident = (rng.standard_normal((r, 1, r)), None, rng.standard_normal((rp, 1, rp)))
    mk = lambda o: P.ProjOp(_cuda(o[0]), None if o[1] is None else _cuda(o[1]), _cuda(o[2]))
    blocks = [P.LocalBlock(0, 0, 1.5, [mk(o1)]),
              P.LocalBlock(1, 0, -0.5, [mk(ident)]),
              P.LocalBlock(1, 1, 2.0, [mk(o2), mk(o3)]),
              P.LocalBlock(0, 1, 1.0, [mk(o3)])]
    K = P.LocalOp(r, rp, 2, blocks, m=m, precision=precision)
    dense = {"o1": o1, "o2": o2, "o3": o3, "id": ident}
    return K, dense


def _dense_K(dense, r, rp, m):
    loc = lambda o: (ott.local_dense(o[0], o[1], o[2]) if o[1] is not None else
                     np.kron(np.kron(o[0][:, 0, :], np.eye(m)), o[2][:, 0, :]))
    p = r * m * rp
    A = np.zeros((2 * p, 2 * p))
    A[:p, :p] += 1.5 * loc(dense["o1"])
    A[p:, :p] += -0.5 * loc(dense["id"])
    A[p:, p:] += 2.0 * loc(dense["o3"]) @ loc(dense["o2"])
    A[:p, p:] += loc(dense["o3"])
    return A


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_local_matvec_twice(precision):
    import paper_2509_11890_amd as P
    rng = np.random.default_rng(7 + precision)
    sizes = [(37, 29, 11, 9), (13, 8, 5, 3)]   # the second call is smaller
    for r, rp, R, R2 in sizes:
        K, dense = _system(P, rng, r, rp, R, R2, precision=precision)
        n = 2 * r * 4 * rp
        x = _cuda(rng.standard_normal(n))
        y_ref = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        y = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        P.local_matvec(K, x, y_ref)
        P.local_matvec_noalloc(K, x, y)
        torch.cuda.synchronize()
        a, b = y.cpu().numpy(), y_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        # same kernels, same launch grouping and summation order
        assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(b), (r, rp, precision)
        if precision == 0:
            ref = _dense_K(dense, r, rp, 4) @ x.cpu().numpy()
            assert np.linalg.norm(a - ref) <= 1e-12 * np.linalg.norm(ref)


def test_noalloc_rejects_oversize_and_launches_nothing():
    import paper_2509_11890_amd as P
    rng = np.random.default_rng(3)
    r, R = 128, 256
    m = 4
    op = P.ProjOp(_cuda(rng.standard_normal((r, R, r))), _cuda(rng.standard_normal((R, m, m, R))),
                  _cuda(rng.standard_normal((r, R, r))))
    K = P.LocalOp(r, r, 1, [P.LocalBlock(0, 0, 1.0, [op])])
    x = _cuda(rng.standard_normal(r * m * r))
    y = torch.full((r * m * r,), 3.25, dtype=torch.float64, device="cuda")
    with pytest.raises(P.TTError) as e:
        P.local_matvec_noalloc(K, x, y)
    assert e.value.code == P.binding.TT_ERR_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(y == 3.25))
