"""The committed tuning table (tile shape per kernel family and degree) is
well formed: the choices only change speed, never results, but a malformed
table must not reach the library."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2004_08503_amd", "tuning_table.json")


def test_table_is_well_formed():
    if not os.path.exists(TABLE):
        pytest.skip("no tuning table")
    with open(TABLE) as f:
        t = json.load(f)
    assert t["tile_shape"]
    with open(os.path.join(ROOT, "include", "idp_dg.h")) as f:
        nshapes = int([l for l in f if l.startswith("#define IDP_DG_NUM_TILE_SHAPES")][0].split()[2])
    for fam, per_p in t["tile_shape"].items():
        assert int(fam) > 0
        for p, shape in per_p.items():
            assert 1 <= int(p) <= 8 and 0 <= shape < nshapes
