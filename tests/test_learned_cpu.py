"""Host-side pieces of the learned decoder (no GPU): k-means recovers
well-separated clusters; the fallback rule; initial weights' layout."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def learned():
    from paper_1705_07272_amd import learned as m
    return m


def test_kmeans_separated_blobs(learned):
    rng = np.random.default_rng(0)
    centres = rng.normal(size=(5, 6)) * 20
    X = np.concatenate([c + rng.normal(size=(200, 6)) for c in centres])
    C, lab = learned.kmeans(X, 5, iters=20, seed=3)
    # every blob maps to exactly one cluster and every cluster to one blob
    blob = np.repeat(np.arange(5), 200)
    pairs = {(b, l) for b, l in zip(blob, lab)}
    assert len(pairs) == 5 and len({l for _, l in pairs}) == 5
    for b in range(5):
        assert np.linalg.norm(C[lab[blob == b][0]] - centres[b]) < 0.5


def test_fallback_rule(learned):
    assert learned.choose_form(9e-4) == "mlp"
    assert learned.choose_form(1e-3) == "mlp"
    assert learned.choose_form(1.1e-3) == "stored"


def test_init_layout(learned):
    w, b = learned.init_weights(0)
    assert w.size == 294912 and b.size == 1280
    first = w[:256 * 128].reshape(256, 128)
    assert abs(first.std() - np.sqrt(2 / 128)) < 0.01
