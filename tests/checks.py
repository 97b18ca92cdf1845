"""Comparison rules of the GPU parity tests (the bar, derived from the FP64
rounding of the two-pass moments and of the QR refit):

  * selected candidate IDs and L0 winners: identical; where the reference
    itself has a near-tie (|delta s| <= 1e-12 s at the cut, not a
    duplicate) either member is accepted;
  * scores: |s_gpu - s_ref| <= 1e-10 s_ref;
  * RMSE: <= 1e-10 relative (+1e-13 std(y) absolute);
  * coefficients: <= 1e-10 relative to the largest |coef| of the model.
"""
import numpy as np

S_RTOL = 1e-10
TIE = 1e-12


def check_selection(g_ids, g_sc, o_ids, o_sc, all_scores=None, what=""):
    """Identical lists up to documented near-ties; scores within S_RTOL."""
    g_ids = [int(i) for i in g_ids if i >= 0]
    o_ids = [int(i) for i in o_ids]
    assert len(g_ids) == len(o_ids), (what, len(g_ids), len(o_ids))
    o_map = dict(zip(o_ids, o_sc))
    g_map = dict(zip(g_ids, g_sc[:len(g_ids)]))
    if set(g_ids) != set(o_ids):
        sk = min(o_sc)
        extra = set(g_ids) - set(o_ids)
        missing = set(o_ids) - set(g_ids)
        for i in missing:
            assert o_map[i] <= sk * (1 + TIE), (what, "missing", i, o_map[i], sk)
        for i in extra:
            assert all_scores is not None and abs(all_scores[i] - sk) <= TIE * sk, (what, "extra", i)
    for a, b in zip(g_ids, o_ids):
        if a != b:
            assert abs(g_map[a] - o_map.get(b, g_map[a])) <= TIE * max(g_map[a], 1e-300) * 10, \
                (what, "order", a, b)
    for i in set(g_ids) & set(o_ids):
        assert abs(g_map[i] - o_map[i]) <= S_RTOL * o_map[i], (what, i, g_map[i], o_map[i])


def check_model(g_sub_ids, g_rmse, g_coef, o_model, y, what=""):
    assert tuple(sorted(g_sub_ids)) == tuple(sorted(o_model["ids"])), (what, g_sub_ids, o_model["ids"])
    assert abs(g_rmse - o_model["rmse"]) <= 1e-10 * o_model["rmse"] + 1e-13 * np.std(y), \
        (what, g_rmse, o_model["rmse"])
    # order coefficients by ID for comparison (both sides: intercept first)
    order_g = np.argsort(g_sub_ids)
    order_o = np.argsort(o_model["ids"])
    cg = np.concatenate([[g_coef[0]], np.asarray(g_coef[1:])[order_g]])
    co = np.concatenate([[o_model["coef"][0]], np.asarray(o_model["coef"][1:])[order_o]])
    scale = np.max(np.abs(co))
    assert np.max(np.abs(cg - co)) <= 1e-10 * scale, (what, cg, co)
