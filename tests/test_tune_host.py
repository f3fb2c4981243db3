"""Host-side checks of the autotuner's bucketing and cache handling."""
import json

from paper_1405_0194_amd import binding as B
from paper_1405_0194_amd import lattice, tune


def test_bucket_is_structural_and_stable():
    s1 = lattice.make_system("cubic", (5, 5, 5), 4, 2.0, 1)
    s2 = lattice.make_system("cubic", (5, 5, 5), 4, 2.0, 2)    # same pattern, other values
    a1, a2 = B.Analysis.from_system(s1), B.Analysis.from_system(s2)
    assert tune.bucket(a1, 40) == tune.bucket(a2, 40)
    assert tune.bucket(a1, 40) != tune.bucket(a1, 80)
    c = lattice.make_system("chain", 2000, 1, 1.0, 1)
    assert tune.bucket(B.Analysis.from_system(c), 40) != tune.bucket(a1, 40)


def test_tuned_options_are_applied(tmp_path):
    s = lattice.make_system("honeycomb", (6, 6), 13, 3.0, 5)
    a = B.Analysis.from_system(s)
    key = tune.bucket(a, 40)
    path = tmp_path / "t.json"
    path.write_text(json.dumps({key: {"options": {"leaf_cols": 64, "panel_width": 32, "tile_rows": 128}}}))
    cache = tune.load_cache(str(path))
    assert tune.options_for(s, 40, cache=cache) == {"leaf_cols": 64, "panel_width": 32, "tile_rows": 128}
    t = tune.tuned_analysis(s, 40, cache=cache)
    assert t.info["npanel"] > a.info["npanel"]          # narrower panels
    assert tune.options_for(s, 80, cache=cache) == tune.DEFAULTS   # untuned bucket


def test_separator_cut_taken_in_3d_not_in_2d():
    # a 3D bulk: the cut removes stored zeros and is taken; a 2D sheet: the
    # separators' columns share their structure and the cut is left out
    cube = lattice.make_system("cubic", (10, 10, 10), 13, 2.0, 7)
    a = tune.with_separator_cut(cube, B.Analysis.from_system(cube))
    assert a.options["sep_cols"] == tune.SEP_COLS
    whole = B.Analysis.from_system(cube)
    assert a.info["nnz_L"] <= (1.0 - tune.CUT_MIN_GAIN) * whole.info["nnz_L"]
    assert a.info["bytes_per_shift"] < whole.info["bytes_per_shift"]
    sheet = lattice.make_system("honeycomb", (20, 20), 13, 3.0, 7)
    b = tune.with_separator_cut(sheet, B.Analysis.from_system(sheet))
    assert b.options["sep_cols"] == 0
    # the tuned analysis applies the same rule
    assert tune.tuned_analysis(cube, 60, cache={}).options["sep_cols"] == tune.SEP_COLS
