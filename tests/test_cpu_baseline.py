"""The multicore CPU timing baseline (oracle/mbbc.c, in the manner of
Algorithm 2) gives the serial oracle's count: tiny random graphs, both side
choices by size, ties, degenerate graphs and a mid-size power-law graph."""
import numpy as np

import oracle
from paper_2601_17707_amd import synth


def test_matches_oracle_on_small_graphs():
    rng = np.random.default_rng(5)
    for _ in range(400):
        g = synth.small_random_graph(rng, max_n=12)
        total, threads = oracle.mbbc_count(g)
        assert total == oracle.count(g)
        assert threads >= 1


def test_matches_oracle_on_power_law_graph():
    for n_u, n_v in ((30_000, 12_000), (12_000, 30_000), (20_000, 20_000)):
        g = synth.chung_lu_graph(n_u, n_v, 200_000, 2.1, 2.1, 2000, 2000, 3, p_neg=0.3)
        assert oracle.mbbc_count(g)[0] == oracle.count(g)


def test_degenerate():
    for n_u, n_v in ((0, 0), (1, 5), (5, 1), (4, 3)):
        e = synth.from_edges(n_u, n_v, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int8))
        assert oracle.mbbc_count(e)[0] == 0
    g = synth.complete_graph(5, 7)
    assert oracle.mbbc_count(g)[0] == 21 * 10
