import os
import sys
import warnings

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def system():
    from paper_2109_00661_amd import workloads as W
    return W.system()


@pytest.fixture(scope="session")
def K_oracle(system):
    from oracle import em
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        return em.make_K(system)


@pytest.fixture(scope="session")
def truth_data(system, K_oracle):
    """Synthetic sounding of the three-layer truth: oracle response plus seeded noise
    scaled by the noise model evaluated at the response."""
    from paper_2109_00661_amd import workloads as W
    from oracle import em
    y = em.forward(W.truth_three_layer(), system, K_oracle)[0]
    s = np.sqrt(em.noise_variance(y, system["eps_an"], system["eps_mn"]))
    return y + s * W.data_noise(1)
