"""The parity harness itself, on the CPU: a box stand-in driven by the oracle
that decides one move differently must be reported as a near-tie and
resynchronised (the oracle's state after that move imported, both chains
continued), and a difference away from a tie must fail."""
import numpy as np
import pytest

from paper_1408_3764_amd import workloads
from tests import helpers


class OracleBox:
    """Stands in for Box: step() runs the oracle chain from the imported state
    and flips the decision of move `flip` (once), as a GPU deciding a near-tie
    the other way would."""

    def __init__(self, orc, pos, p, seed, max_n, flip):
        self.orc, self.p, self.seed, self.max_n, self.flip = orc, p, seed, max_n, flip
        self.pos = pos.copy()
        self.imports = []

    def step(self, n_moves, counter0=0, log=False):
        pos, _, lg = self.orc.chain(self.pos, n_moves, self.p, seed=self.seed, counter0=counter0, max_n=self.max_n)
        lg = lg.copy()
        k = self.flip - counter0
        if 0 <= k < n_moves:
            lg["accepted"][k] = 1 - lg["accepted"][k]
            self.flip = -1
        self.pos = pos
        return None, lg

    def import_state(self, pos, ck):
        self.pos = np.asarray(pos).copy()
        self.imports.append(int(ck["counter"]))


def _setup(orc):
    wb = workloads.random_box(120, 7.0, seed=8, T=1.2)
    p = orc.make_params(wb.L, 2.5, beta=1 / 1.2, mu=-2.0)
    return wb, p


def test_near_tie_is_recorded_and_resynchronised(orc, monkeypatch):
    wb, p = _setup(orc)
    _, _, olog = orc.chain(wb.pos, 400, p, seed=3, max_n=700)
    flip = int(np.nonzero((olog["flags"] & 1) == 0)[0][150])
    monkeypatch.setattr(helpers, "near_tie", lambda o, beta: True)
    box = OracleBox(orc, wb.pos, p, 3, 700, flip)
    r = helpers.chain_parity(box, orc, wb.pos, p, 3, 400, 1 / 1.2, 700, "stand-in")
    assert r["ties"] == [flip]
    assert box.imports == [flip + 1]
    assert np.array_equal(box.pos, r["opos"])


def test_difference_away_from_a_tie_fails(orc):
    wb, p = _setup(orc)
    box = OracleBox(orc, wb.pos, p, 3, 700, 57)
    with pytest.raises(AssertionError, match="away from a tie"):
        helpers.chain_parity(box, orc, wb.pos, p, 3, 400, 1 / 1.2, 700, "stand-in")
