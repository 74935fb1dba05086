"""The launch shapes kept for the FV 2048 x 2048 FP64 solve (the ones the
benchmark and the full-size parity test pin) are well formed: every entry
names a solve operator once, with a shape that airg_set_lanes accepts
(lanes 0 or a power of two up to 64, XCD mapping 0 or 1, LDS staging 0, 1
with 2 to 16 lanes, or 2 with one lane), and the levels cover the hierarchy
the solve builds (nine levels, the coarsest level's matrix once)."""
from paper_2508_17517_amd import load_shapes

OPS = {"ff", "b", "z", "a", "top"}
LANES = {0, 1, 2, 4, 8, 16, 32, 64}


def test_fv2048_shapes_are_well_formed():
    shapes = load_shapes("fv2048_fp64")
    assert shapes, "no shapes kept"
    seen = set()
    for e in shapes:
        assert {"level", "op", "lanes", "xcd_map", "lds"} <= set(e), e
        assert e["op"] in OPS, e
        assert isinstance(e["level"], int) and e["level"] >= 0, e
        assert e["lanes"] in LANES, e
        assert e["xcd_map"] in (0, 1), e
        assert e["lds"] in (0, 1, 2), e
        if e["lds"] == 1:
            assert 2 <= e["lanes"] <= 16, e
        if e["lds"] == 2:
            assert e["lanes"] == 1, e
        key = (e["op"], None if e["op"] in ("a", "top") else e["level"])
        assert key not in seen, e
        seen.add(key)
    assert ("a", None) in seen and ("top", None) in seen
    # the operators of every level above the coarsest: A_ff, B and Z
    coarsest = next(e["level"] for e in shapes if e["op"] == "a")
    assert coarsest == 8
    for lvl in range(coarsest):
        for op in ("ff", "b", "z"):
            assert (op, lvl) in seen, (op, lvl)
    assert len(shapes) == 3 * coarsest + 2
