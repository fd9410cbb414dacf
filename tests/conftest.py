import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def model_path():
    from synth import default_model_file
    return default_model_file()


@pytest.fixture(scope="session")
def omodel(model_path):
    from oracle import load_model
    return load_model(model_path)


@pytest.fixture(scope="session")
def water192():
    from synth import config_system
    return config_system("water192")


@pytest.fixture(scope="session")
def oracle_water192(omodel, water192):
    from oracle.dp import evaluate
    s = water192
    return evaluate(omodel, s.coords, s.types, s.box)


def _gpu_model(model_path, precision):
    from paper_2602_02234_amd import Model
    return Model(model_path, precision=precision)


@pytest.fixture(scope="session")
def gpu_fp32(model_path):
    return _gpu_model(model_path, "fp32")


@pytest.fixture(scope="session")
def gpu_bf16(model_path):
    return _gpu_model(model_path, "bf16")


@pytest.fixture(scope="session")
def gpu_models(gpu_fp32, gpu_bf16):
    return {"fp32": gpu_fp32, "bf16": gpu_bf16}


@pytest.fixture(autouse=True)
def _announce(request):
    """Name each test before it runs (flushed), so a run cut short still shows where it was."""
    import sys
    sys.stdout.write(f"\n[start] {request.node.nodeid}\n")
    sys.stdout.flush()
    yield
