"""Volume changes (the cell-list rebuild and total energy that Gibbs-ensemble
volume moves need, Sec. 5 of the paper) against the oracle: coordinates scaled
bit for bit, the rebuilt grid and cell assignment bit-exact, the cell-list
energies at both volumes within the energy tolerance, and the chain after the
change identical to the oracle's chain from the scaled configuration."""
import numpy as np
import pytest

import oracle
from paper_1408_3764_amd import workloads
from tests.helpers import compare_chain_logs

pytestmark = pytest.mark.gpu


def _params(wb, L):
    return oracle.make_params(L, wb.rc, eps=wb.eps, sigma=wb.sigma, beta=wb.beta, mu=wb.mu,
                              lambda3=wb.lambda3, max_disp=wb.max_disp, p_disp=wb.p_disp)


def _scaled(pos, L, L_new):
    """x -> x * (L'/L), the ratio rounded once, kept in [0, L')."""
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    L_new = np.broadcast_to(np.asarray(L_new, dtype=np.float64), (3,))
    y = pos * (L_new / L)
    y = np.where(y >= L_new, y - L_new, y)
    return np.where(y >= L_new, 0.0, y)


@pytest.mark.parametrize("lam,cm", [([1.03] * 3, None), ([0.96] * 3, None), ([1.02, 0.97, 1.05], None),
                                    ([0.9] * 3, None), ([1.04] * 3, [16, 16, 16])])
def test_rescale_matches_oracle(lam, cm):
    from paper_1408_3764_amd.box import Box
    wb = workloads.small()
    b = Box.from_workload(wb, max_n=wb.n + 10, cell_m=cm)
    L_new = wb.L * np.array(lam)
    got = b.rescale(L_new)
    ref_old = oracle.total_energy(wb.pos, _params(wb, wb.L))
    q = _scaled(wb.pos, wb.L, L_new)
    ref = oracle.total_energy(q, _params(wb, L_new))
    assert abs(got["U_pair_old"] - ref_old["U_pair"]) <= 1e-10 * ref_old["sumabs"]
    assert abs(got["U_pair"] - ref["U_pair"]) <= 1e-10 * ref["sumabs"]
    assert got["U_tail"] == pytest.approx(ref["U_tail"], rel=1e-13)
    assert got["U_tail_old"] == pytest.approx(ref_old["U_tail"], rel=1e-13)
    pos, _ = b.particles()
    assert np.array_equal(pos, q)
    req = None if cm is None else np.array(cm, dtype=np.int32)
    g = oracle.grid(L_new, wb.rc, req)
    info = b.info()
    assert info["cell_m"] == list(g["M"]) and info["span"] == list(g["span"])
    assert info["n_stencil"] == oracle.stencil_count(L_new, wb.rc, req)
    cell_of, count, _ = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(q, L_new, wb.rc, req))
    assert count.max() <= info["cell_cap"]


def test_rescale_grid_changes_and_chain_continues():
    """Compressing L = 20 to 19.5 drops the grid from 8 to 7 cells per axis; the
    chain after the change is the oracle's chain from the scaled configuration,
    and the running energy is the new total."""
    from paper_1408_3764_amd.box import Box
    wb = workloads.small()
    b = Box.from_workload(wb, max_n=wb.n + 400)
    assert b.info()["cell_m"] == [8, 8, 8]
    L_new = np.array([19.5, 19.5, 19.5])
    got = b.rescale(L_new)
    assert b.info()["cell_m"] == [7, 7, 7]
    assert b.checkpoint()["u_pair"] == got["U_pair"]
    q = _scaled(wb.pos, wb.L, L_new)
    p = _params(wb, L_new)
    _, _, olog = oracle.chain(q, 300, p, seed=wb.seed, max_n=wb.n + 400, U0=0.0)
    for shape in [(4, 4), (8, 0)]:
        c = Box.from_workload(wb, max_n=wb.n + 400)
        c.rescale(L_new)
        c.set_launch(*shape)
        _, glog = c.step(300, counter0=0, log=True)
        assert compare_chain_logs(glog, olog, wb.beta) == 300, shape
        c.close()


def test_rescale_round_trip_and_errors():
    from paper_1408_3764_amd.box import Box
    from paper_1408_3764_amd._lib import GcmcError
    wb = workloads.small()
    b = Box.from_workload(wb, max_n=wb.n + 10)
    before = b.particles()[0]
    info0 = b.info()
    with pytest.raises(GcmcError):
        b.rescale([4.9, 20.0, 20.0])          # rc > L/2
    assert np.array_equal(b.particles()[0], before) and b.info() == info0
    r1 = b.rescale(wb.L * 1.05)
    r2 = b.rescale(wb.L)
    assert np.allclose(b.particles()[0], before, rtol=0, atol=1e-13 * wb.L[0])
    assert r2["U_pair"] == pytest.approx(r1["U_pair_old"], rel=1e-9)
