"""The seeded input generators (CPU only): shapes, determinism and the
structure each dataset is meant to have."""
import numpy as np
import pytest

from paper_2106_13706_amd import workloads


@pytest.mark.parametrize("name", workloads.POWER_DATASETS)
def test_power_datasets_shapes_and_seeds(name):
    P, Q = workloads.power_dataset(name, 37, d=4, seed=5)
    assert P.shape == (37, 4) and Q.shape == (37, 4)
    assert P.dtype == np.float32 and Q.dtype == np.float32
    P2, Q2 = workloads.power_dataset(name, 37, d=4, seed=5)
    assert (P == P2).all() and (Q == Q2).all()
    P3, _ = workloads.power_dataset(name, 37, d=4, seed=6)
    assert not (P == P3).all()
    assert np.isfinite(P).all() and np.isfinite(Q).all()


def test_power_dataset_structure():
    P, Q = workloads.power_dataset("DVU", 500)
    assert (P == P[:, :1]).all()  # the diagonal
    assert P.min() >= 0 and P.max() <= 1 and Q.min() >= 0 and Q.max() <= 1
    P, Q = workloads.power_dataset("Skew", 2000)
    assert P.min() > 0 and Q.min() > 0 and Q.mean() < P.mean()  # the larger rate
    P, Q = workloads.power_dataset("MM", 1000, delta=0.0, noise=0.25)
    assert (np.abs(P[:250]) <= 3).all() and (np.abs(Q[:250]) <= 3).all()  # the noise part
    assert np.abs(P[:250]).max() > 2.9 and np.abs(P[250:]).max() > 3
    P, Q = workloads.power_dataset("GVS", 4000, delta=1.0)
    assert abs(Q.std() / P.std() - 2.0) < 0.1
    P, Q = workloads.power_dataset("GVM", 4000, delta=1.0)
    assert abs(Q.mean() - P.mean() - 1.0) < 0.1
    with pytest.raises(ValueError):
        workloads.power_dataset("LS", 10)


def test_serving_stream_materialize_matches():
    s1 = workloads.serving_stream(n_requests=20, materialize=True)
    s2 = workloads.serving_stream(n_requests=20, materialize=False)
    for a, b in zip(s1.requests, s2.requests):
        P, Q = workloads.materialize(b)
        assert (P == a.P).all() and (Q == a.Q).all() and a.d == b.d
