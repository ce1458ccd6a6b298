"""The stored full-size results (tests/golden/) against the generators and
the oracle, on the CPU: the graphs the GPU tests and the benchmark build are
the graphs the results were written for, and the oracle still produces
them. Their certification by independent algorithms (the Johnson closed
form, Dijkstra, the planted cycle) happens in tests/golden/make_golden.py
before anything is written."""
import numpy as np
import pytest

import goldens
import oracle
import synth


def test_grid64_matches_oracle_and_generator():
    g = synth.config_graph("grid64")
    rec = goldens.load("grid64")
    assert goldens.graph_digest(g) == rec["graph_sha256"]
    d, p, neg = oracle.sssp(g, method="rounds")
    assert not neg
    goldens.check(rec, d, p, "grid64")
    assert rec["certified_by"] == "dijkstra"


@pytest.mark.slow
def test_rmat20_matches_oracle_and_generator():
    g = synth.config_graph("rmat20")
    rec = goldens.load("rmat20")
    assert goldens.graph_digest(g) == rec["graph_sha256"]
    d, p, neg = oracle.sssp(g, method="fifo")
    assert not neg
    goldens.check(rec, d, p, "rmat20")
    assert rec["m_reached"] == int(np.diff(g.offsets)[d != oracle.INF].sum())
    x = goldens.load("rmat20_x64_sources")
    srcs = synth.random_sources(g, 64, seed=x["sources_seed"])
    assert [q["src"] for q in x["queries"]] == [int(s) for s in srcs]
    # two of the 64 batched sources, recomputed
    for q in (x["queries"][0], x["queries"][63]):
        d, p, neg = oracle.sssp(g, q["src"], method="fifo")
        goldens.check(q, d, p, f"rmat20 src={q['src']}")


@pytest.mark.slow
def test_road2048_generators_match():
    for name in ("road2048", "road2048_negcycle"):
        g = synth.config_graph(name)
        rec = goldens.load(name)
        assert goldens.graph_digest(g) == rec["graph_sha256"], name
        assert (name == "road2048_negcycle") == rec["neg_cycle"]


@pytest.mark.slow
def test_er256_matches_oracle_and_generator():
    x = goldens.load("er256")
    graphs = synth.er_batch(256)
    assert x["count"] == len(x["queries"]) == len(graphs) == 256
    for g, q in zip(graphs, x["queries"]):
        assert goldens.graph_digest(g) == q["graph_sha256"], g.name
        assert g.src == q["src"] and g.n == q["n"] and g.m == q["m"]
    # the smallest and the largest instance, recomputed
    sizes = [g.n for g in graphs]
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        g, q = graphs[i], x["queries"][i]
        d, p, neg = oracle.sssp(g, g.src, method="fifo")
        assert not neg
        goldens.check(q, d, p, g.name)
        assert q["m_reached"] == int(np.diff(g.offsets)[d != oracle.INF].sum())
