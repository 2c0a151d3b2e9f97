"""The paper's stated parameters (Sec. III) against the oracle's index set."""

import json
import os

import numpy as np

from oracle import basis

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_bands_are_nested_prefixes():
    p = json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))
    L_max = p["L_max"]["value"]
    idx = basis.IndexSet(L_max)
    sizes = [idx.prefix(L) for L in p["L_set"]["value"]]
    assert sizes == sorted(sizes) and sizes[-1] < idx.size
    for L, n in zip(p["L_set"]["value"], sizes):
        assert np.all(idx.l[:n] <= L)
        assert n == basis.IndexSet(L).size
    assert p["lowest_band_for_candidates"]["value"] == min(p["L_set"]["value"])
