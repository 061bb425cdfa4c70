"""What the trained network gains, measured end to end on the GPU.

Trains the proposal's network with the library's kernels on 1e5 injections
and 1e5 noise draws that the method itself generates (the workload of the
learned-proposal configuration: 256 coarse chirp-mass cells x 20 sub-bands,
120 segments of 30 s at 256 Hz, SNR uniform 4-20), with early stopping on a
held-back tenth, then checks:

- held-out discrimination of injection regions from noise (fresh windows,
  5120 of each): the trained network's ROC AUC beats the region's own
  largest coarse z (the non-learned score, which is one of its 64 inputs) and
  far exceeds its untrained initialisation;
- the search: refining only the network's top 512 of the 5120 regions (a 10x
  cut of the fine-grid cost) loses at most 1 % of the injections that the
  exhaustive fine search detects, and no more than ranking by the largest
  coarse z loses at the same k (2048 held-out injections, threshold at a
  1 % false-alarm probability of the exhaustive search over 1000 noise draws).

The full-scale run of the same procedure (20,000 held-out injections) is the
committed result of ``python -m paper_2609_12476_amd.proposal_experiment``.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_trained_network_gains_over_max_z_and_exhaustive(gpu):
    from paper_2609_12476_amd import proposal_experiment as pe
    print("learned proposal gain (trains on the GPU)", flush=True)
    r = pe.run(scale=1.0, n_mc=256, per_cell=8, ks=(512,), epochs=30, seed=1234, n_judge=2048,
               thr_draws=1000, quiet=True)
    k512 = r["by_k"][0]
    print({k: r[k] for k in ("heldout_auc_learned", "heldout_auc_max_z", "heldout_auc_untrained",
                             "detected_exhaustive", "total_seconds")}, k512, flush=True)
    sys.stdout.flush()
    assert r["heldout_auc_learned"] >= r["heldout_auc_max_z"] + 0.002
    assert r["heldout_auc_learned"] >= r["heldout_auc_untrained"] + 0.3
    assert r["detected_exhaustive"] >= 200
    assert k512["refined_fraction"] == pytest.approx(0.1)
    assert k512["lost_of_exhaustive_detections_learned"] <= 0.01
    assert k512["lost_of_exhaustive_detections_learned"] <= k512["lost_of_exhaustive_detections_baseline"]
