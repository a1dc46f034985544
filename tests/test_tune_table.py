"""The tuning table's lookups, no GPU: a Problem's shape is the entry's fastest
candidate; a served request's is the fastest candidate with strips of at least
SERVED_MIN_ROWS rows (one-row strips pay off only for a grid alone on the chip);
the committed table resolves for every tuned energy, precision and size class."""
from paper_1604_06525_amd import tune

ENTRY = {"energy": "arap_warp", "precision": "mixed", "min_sites": 8192, "max_sites": 32768, "side": 128,
         "strip_rows": 1, "waves_per_simd": 0, "iter_us": 7.0,
         "candidates": {"rows=1": 7.0, "rows=2": 7.9, "rows=4": 9.8, "rows=6": 11.1, "waves=1": 9.7,
                        "waves=2": 9.65, "auto=0": 9.66}}


def test_solo_takes_the_fastest_candidate():
    assert tune.choice(ENTRY) == {"strip_rows": 1, "waves_per_simd": 0}
    assert tune.best([ENTRY], "arap_warp", "mixed", 16384) == {"strip_rows": 1, "waves_per_simd": 0}


def test_served_skips_short_strips():
    assert tune.choice(ENTRY, served=True) == {"strip_rows": 0, "waves_per_simd": 2}
    assert tune.best([ENTRY], "arap_warp", "mixed", 16384, served=True) == {"strip_rows": 0, "waves_per_simd": 2}
    tall = dict(ENTRY, strip_rows=6)
    assert tune.choice(tall, served=True) == {"strip_rows": 6, "waves_per_simd": 0}
    bare = dict(ENTRY, candidates={"rows=1": 7.0})
    assert tune.choice(bare, served=True) == {"strip_rows": tune.SERVED_MIN_ROWS, "waves_per_simd": 0}


def test_no_entry_keeps_the_library_choice():
    assert tune.best([ENTRY], "arap_warp", "fp64", 16384) == {"strip_rows": 0, "waves_per_simd": 0}
    assert tune.best([ENTRY], "arap_warp", "mixed", 100) == {"strip_rows": 0, "waves_per_simd": 0}


def test_committed_table_resolves():
    entries = tune.load()
    assert entries
    for e in entries:
        for served in (False, True):
            c = tune.choice(e, served)
            assert c["strip_rows"] >= 0 and c["waves_per_simd"] >= 0
            if served and c["strip_rows"]:
                assert c["strip_rows"] >= tune.SERVED_MIN_ROWS
