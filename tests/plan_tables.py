"""The oracle's own view of a plan (test helper).

Everything the oracle is given about a plan comes from the arguments the test passed to
the library (kept by the binding as `Plan.args`), never from the library's outputs: the
DM trials from `oracle.dm_trials`, the delay table from `oracle.delay_table` (Eq. (1)),
the block sizes from `oracle.sizes`.  A plan made from an explicit delay table keeps the
test's own table (its DM values default to the trial index, as the header states).
`assert_library_tables` then checks the library's own tables against these, separately.
"""
import numpy as np

import oracle


def oracle_plan(plan) -> dict:
    a = plan.args
    if a["delays"] is not None:
        D = np.asarray(a["delays"], np.int64)
        dms = np.arange(D.shape[0], dtype=np.float64) if a["dms"] is None else np.asarray(a["dms"], np.float64)
    else:
        dms = oracle.dm_trials(a["dm_ranges"])
        D, _ = oracle.delay_table(a["nchans"], a["fch1"], a["foff"], a["tsamp"], dms)
    sz = oracle.sizes(D, a["n_out"], a["widths"])
    L = a["norm_window"] if a["norm_window"] > 0 else a["n_out"]
    return {"D": D, "dms": dms, "n_out": a["n_out"], "L": L, "widths": a["widths"], "threshold": a["threshold"],
            "stencils": a["stencils"], "tsamp": a["tsamp"], "nchans": a["nchans"], "fch1": a["fch1"],
            "foff": a["foff"], **sz}


def assert_library_tables(plan) -> dict:
    """The library's delay table, DM values and block sizes equal the oracle's."""
    o = oracle_plan(plan)
    assert np.array_equal(plan.delays().astype(np.int64), o["D"]), "library delay table differs from the oracle's"
    assert np.array_equal(plan.dms(), o["dms"]), "library DM values differ from the oracle's"
    i = plan.info
    assert (i["s_max"], i["n_dd"], i["n_in"]) == (o["s_max"], o["n_dd"], o["n_in"])
    return o


def search_beam(plan, x, beam=0) -> dict:
    """oracle.search_beam on the oracle's own view of the plan."""
    o = oracle_plan(plan)
    return oracle.search_beam(x[:, :o["n_in"]], o["D"], o["dms"], o["n_out"], o["L"], o["widths"], o["threshold"],
                              stencils=o["stencils"], beam=beam)
