"""The paper's printed path counts for full QUAPI (Sec. 4.2) against the
stored-set size of the oracle, which reaches M^(2 dk_max) at small dk_max."""
import json
import os

import numpy as np

import oracle
from oracle.eta import Bath, eta_columns
from paper_2506_03127_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_printed_counts_are_m_to_the_2k(oracle_mod):
    g = json.load(open(os.path.join(HERE, "golden", "paper_path_counts.json")))
    M = g["M"]
    for row in g["printed"]:
        exact = M ** (2 * row["dk_max"])
        assert f"{exact:.1e}" == f"{row['paths']:.1e}"
    # the oracle's stored set at small dk_max follows the same law
    for K in (2, 3, 4):
        eta = eta_columns(Bath(0.1, 5.0), 5.0, 0.25, K)
        o = oracle.Oracle(W.tls_hamiltonian(0.0, 1.0), [1, -1], 0.25, K, eta,
                          W.ground_projector(2), mode=oracle.POST)
        o.step(K + 1)
        assert o.stats(K + 1)["n_stored"] == M ** (2 * K)
