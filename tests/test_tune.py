"""The autotuner's table (paper_2310_18043_amd/tuned.json) and its lookup, on the CPU."""
import json
import os

from paper_2310_18043_amd import tune
from paper_2310_18043_amd import workloads as W


def test_table_entries_are_well_formed():
    table = tune.load_table()
    assert table, "tuned.json is missing or empty"
    for key, e in table.items():
        assert key.startswith("n=") and "precision=" in key
        assert e["tile"] in (16, 32, 64, 128, 256)
        # eight columns per workgroup exist at tile 256 only
        assert e["trsm_cols"] in ((1, 2, 4, 8) if e["tile"] == 256 else (1, 2, 4))
        assert e["subblock"] in (1, 2, 4, 8, 16, 32)
        # the chosen entry is the fastest converged candidate it records
        ok = [c for c in e["candidates"] if c["converged"]]
        assert min(c["ms"] for c in ok) == e["ms"]
        assert any(c["tile"] == e["tile"] and c["trsm_cols"] == e["trsm_cols"] and
                   c["subblock"] == e["subblock"] for c in ok)


def test_lookup_matches_the_benchmark_shape_only():
    wl = W.convdiff_workload()
    e = tune.lookup(wl.A, wl.B, wl.p, wl.q, wl.w, 0)
    assert e is not None and e["workload"] == "convdiff128"
    assert tune.lookup(wl.A, wl.B, wl.p, wl.q, 64, 0) is None        # another block width
    assert tune.lookup(wl.A, wl.B, wl.p, wl.q, wl.w, 1) is None      # no precision-form entry


def test_shape_key_uses_the_band_extents():
    wl = W.convdiff_workload()
    kl, ku = tune.bandwidths(wl.A, wl.B)
    assert (kl, ku) == (128, 128)
    assert tune.shape_key(wl.n, kl, ku, 4, 8, 128, 0) == "n=16384,kl=128,ku=128,p=4,q=8,w=128,precision=0"
