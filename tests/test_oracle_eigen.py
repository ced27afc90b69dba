"""The eigenvector-placement oracle (oracle/eigen.py) against closed forms
and scipy's connected components, and plausible mistakes planted in a copy of
it caught by those pins (no GPU).  The real module is never modified."""
import importlib.util
import os
import tempfile

import pytest

from oracle import eigen as E

from oracle_pins import EIGEN_PINS


@pytest.mark.parametrize("pin", EIGEN_PINS, ids=[p.__name__ for p in EIGEN_PINS])
def test_eigen_pin(pin):
    pin(None, E)


MUTANTS = {
    "laplacian_without_degree": ("lap[pos[a], pos[a]] += w", "lap[pos[a], pos[a]] += 0.0"),
    "zero_eigenvalue_kept": ("v = vec[:, 1 + q]", "v = vec[:, q]"),
    "labels_take_largest_index": ("parent[max(ra, rb)] = min(ra, rb)",
                                  "parent[min(ra, rb)] = max(ra, rb)"),
    "weight_models_swapped": ("return 2.0 / m if weight_model == 1 else 1.0 / (m - 1)",
                              "return 1.0 / (m - 1) if weight_model == 1 else 2.0 / m"),
    "smallest_component_picked": ("key=lambda l: (-counts[l], l)", "key=lambda l: (counts[l], l)"),
    "sign_not_fixed": ("if v[int(np.argmax(np.abs(v)))] < 0:", "if False:"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_eigen_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(E.__file__).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "eigen_mutant.py")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        spec = importlib.util.spec_from_file_location("eigen_mutant", path)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        caught = []
        for pin in EIGEN_PINS:
            try:
                pin(None, mod)
            except Exception as exc:  # any failed pin counts
                caught.append((pin.__name__, type(exc).__name__))
        assert caught, f"no pin catches mutant {name}"
