"""The parameters the paper prints that the synthetic workloads rest on
(tests/golden/paper_parameters.json, each with its citation).  The paper
prints no worked example of the facet sum, so no stored output is compared
here; these checks keep the workloads tied to the printed values."""
import json
import math
import os

import numpy as np

import workloads as W
import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "paper_parameters.json")


def load():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_every_entry_cites_the_paper():
    d = load()
    for k, v in d.items():
        if k.startswith("_"):
            continue
        assert "cite" in v and v["cite"].startswith(("Sec.", "Fig.")), k


def test_formation_and_channels():
    d = load()
    lo, hi = d["formation_distance_km"]["min"], d["formation_distance_km"]["max"]
    assert lo <= W.RX_LEAD / 1e3 <= hi
    g = W.harmony_geometry(8, 64, receivers="AB", n_pc=d["harmony_phase_centres"]["value"])
    ch = d["receiving_channels_in_timing_runs"]
    # the Harmony channels of the timing runs; Sentinel-1's own monostatic
    # channel is not part of the bistatic workloads
    assert g.n_channels == 2 * ch["per_harmony"] == ch["value"] - ch["sentinel1"]
    # receivers A and B lead and follow the transmitter by the same distance
    xs = sorted(p.p0[0] - g.platforms[0].p0[0] for p in g.platforms[1:])
    assert xs == [-W.RX_LEAD, W.RX_LEAD]


def test_printed_tiling_weight_is_the_oracle_weight():
    """Eq. 2's printed weight against the oracle's tiled sea: at points of a
    tile, with one node's height set and the others zero, the oracle's field
    is W_q times that node's own field, W_q from the printed form (a
    cross-check of the fixture; the tiling's pins, which do not retype the
    formula, are the corner, energy and variance tests of the sea tiles)."""
    d = load()
    assert "1 - w_x^i - w_y^i + w_x^i w_y^i" in d["tiling_weight"]["form"]
    sea = W.hetero_sea(121, 121, 5.0, 3, 150.0, cwm=False)
    n1 = sea.ntx + 1
    q = 2 * n1 + 1                         # a corner node of tile (1, 2)
    hs = np.zeros_like(sea.node_hs)
    hs[q] = sea.node_hs[q]
    from dataclasses import replace
    only = replace(sea, node_hs=hs)
    own = replace(sea, mode=1, hs=float(sea.node_hs[q]), dirs=sea.node_dirs[q],
                  phases=sea.node_phases[q])
    f = O.generate_facets(only, 3)
    g = O.generate_facets(own, 3)
    xq = sea.tile_x0 + (q % n1) * sea.tile_L
    yq = sea.tile_y0 + (q // n1) * sea.tile_L
    X = (np.arange(121) - 60) * 5.0
    for ix, iy in ((32, 62), (35, 70), (40, 80), (33, 88)):
        wx, wy = abs(X[ix] - xq) / sea.tile_L, abs(X[iy] - yq) / sea.tile_L
        w_printed = math.sqrt(1 - wx - wy + wx * wy)
        p = iy * 121 + ix
        assert abs(f["z"][p] - w_printed * g["z"][p]) < 1e-12 * max(1.0, abs(g["z"][p]))
