"""The seeded synthetic workloads (no method arithmetic): their stated recipe.

The batched-box workload's one deliberate difference from the 256^3 one is the
heat release of its network; its rate draws, species and stoichiometry are the
same, so its Newton-count spread comes from that knob alone.
"""
import numpy as np

import sdc_inputs as si


def test_box_network_differs_from_the_3d_one_only_in_heat_release():
    boxes = si.boxes_workload(nbox=4, choices=(4,))
    net3d = si.workload("net3d", shape=(4, 4, 4))
    a, b = boxes["network"], net3d["network"]
    for key in ("nspec", "nreact"):
        assert a[key] == b[key]
    for key in ("reactants", "stoich", "lnA", "b", "E"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_allclose(a["q"], b["q"] * (0.85 / 0.25), rtol=1e-15)
    assert boxes["node_type"] == "radau" and boxes["n_nodes"] == 3 and boxes["n_iters"] == 4


def test_box_extents_and_offsets():
    w = si.boxes_workload(nbox=64, choices=(8, 16, 32, 64))
    ext, off = np.asarray(w["box_n"]), np.asarray(w["box_off"])
    assert ext.shape == (64, 3) and set(np.unique(ext)) <= {8, 16, 32, 64}
    assert off[0] == 0 and np.array_equal(np.diff(off), np.prod(ext, axis=1))
    assert w["U0"].shape == (18, off[-1])
    # isobaric lognormal temperature: rho = 1 / T with log T = 0.3 zeta
    rho = w["U0"][0]
    logT = -np.log(rho)
    assert abs(np.std(logT) - 0.3) < 0.01 and abs(np.mean(logT)) < 0.01
