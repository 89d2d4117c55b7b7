"""The experiment grids against the parameter values of Table I
(tests/golden/table1_parameters.json, the values as the paper prints them)."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_parameters.json")


def _table1():
    with open(GOLDEN) as f:
        return json.load(f)


def test_table1_pn_lengths_are_m_sequence_periods():
    # Eq. 1: an m-sequence of degree d has period 2^d - 1
    for m in _table1()["pn_sequence_length"]:
        d = m.bit_length()
        assert (1 << d) - 1 == m


def test_latency_sweeps_cover_table1():
    """Figs. 6-7: every MIMO scale, PN length and N_batch of Table I is a
    point; the cyclic prefix (C = L) and the taps lie in Table I's ranges;
    each array splits into whole multiplexed blocks."""
    import bench
    t = _table1()
    pts = bench.LATENCY_POINTS
    assert {n for n, _, _, _ in pts} == set(t["mimo_scale"])
    assert {m for _, m, _, _ in pts} == set(t["pn_sequence_length"])
    assert {nb for _, _, _, nb in pts} == set(t["n_batch"])
    cp_lo, cp_hi = t["cp_length_range"]
    tap_lo, tap_hi = t["channel_taps_range"]
    for n, m, L, nb in pts:
        assert cp_lo <= L <= cp_hi and tap_lo <= L <= tap_hi
        assert n % nb == 0
    # Fig. 6: the sweep over M at 16 x 16 takes every N_batch at every M
    assert {(m, nb) for n, m, L, nb in pts if n == 16 and L == 64} == \
        {(m, nb) for m in t["pn_sequence_length"] for nb in t["n_batch"]}


def test_accuracy_sweeps_within_table1():
    """Figs. 4-5: the curves' PN lengths, N_batch, taps and realisations per
    point are Table I's."""
    from paper_2206_05506_amd import sweeps
    t = _table1()
    tap_lo, tap_hi = t["channel_taps_range"]
    for M, nb, L, lnz in sweeps.FIG4_CURVES + sweeps.FIG5_CURVES:
        assert M in t["pn_sequence_length"] and nb in t["n_batch"]
        assert tap_lo <= lnz <= L <= tap_hi
        assert sweeps.N_T % nb == 0
    assert sweeps.N_T in t["mimo_scale"] and sweeps.N_R == sweeps.N_T
    assert sweeps.DEFAULT_ITERS == t["iterations_per_experiment"]
