"""Host logic of the launch-shape rules (no GPU): which box gets which shape."""
from paper_1408_3764_amd import tune


class FakeBox:
    def __init__(self, n, n_stencil=27, n_cells=27, ns=1):
        self.n = n
        self._info = {"n_species": ns, "n_stencil": n_stencil, "n_cells": n_cells}
        self.launch = None

    def info(self):
        return self._info

    def set_launch(self, waves, rows):
        self.launch = (waves, rows)


def test_lds_rule_holds_small_boxes_and_applies_the_inner_rule_to_the_rest():
    boxes = [FakeBox(300), FakeBox(512), FakeBox(513), FakeBox(20000, n_cells=2197), FakeBox(400, ns=2)]
    rule = ("lds", ((300, (4, -3)), (512, (8, -3))), ("uniform", (4, 0)))
    shapes = tune.apply_batch_rule(boxes, rule)
    # the two-species box cannot take the speculative kernel either: per-move 4x4
    assert [b.launch for b in boxes] == [(4, -3), (8, -3), (4, 0), (4, 0), (4, 4)]
    assert shapes[:4] == [(4, -3), (8, -3), (4, 0), (4, 0)]
    assert tune.rule_name(rule) == "lds300:4x-3,512:8x-3+4x0"


def test_cost_rule_ranks_by_candidates_per_move():
    # a small box whose stencil covers it reads all its particles per move; a large one reads
    # n x 27 / cells
    small_dense = FakeBox(700, n_stencil=27, n_cells=27)
    large = FakeBox(20000, n_stencil=27, n_cells=2197)
    mid = FakeBox(3000, n_stencil=27, n_cells=216)
    boxes = [large, small_dense, mid, FakeBox(200)]
    tune.apply_batch_rule(boxes, ("cost", 0.25, (8, 0), (2, 0)))
    assert small_dense.launch == (8, 0)
    assert large.launch == (2, 0) and mid.launch == (2, 0)
    assert tune.rule_name(("cost", 0.25, (8, 0), (2, 0))) == "cost0.25:8x0/2x0"


def test_every_batch_rule_has_a_name_and_applies():
    boxes = [FakeBox(n, n_cells=max(27, n // 10)) for n in (150, 600, 1500, 5000, 30000)]
    names = set()
    for rule in tune.BATCH_RULES:
        shapes = tune.apply_batch_rule(boxes, rule)
        assert len(shapes) == len(boxes) and all(b.launch is not None for b in boxes)
        names.add(tune.rule_name(rule))
    assert len(names) == len(tune.BATCH_RULES)
