"""The FP64 oracle against what the paper and mathematics fix (CPU only)."""
import os
import subprocess

import pytest

import oracle_pins as P
from oracle import oracle as O


@pytest.fixture(scope="module")
def orc():
    return O.load()


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


# Each planted slip (see PLANT in oracle.c) must be caught by at least one pin.
PLANTS = {
    1: "off-diagonal Gram entries perturbed",
    2: "minus sign of h dropped",
    3: "scale by H_ii instead of sqrt(H_ii)",
    4: "wrong sign in the passive-set test",
    5: "half the exact line-search step",
    6: "plus sign in the projected update",
}


@pytest.mark.parametrize("plant", sorted(PLANTS), ids=lambda p: PLANTS[p].replace(" ", "_"))
def test_pins_catch_planted_mistake(plant, tmp_path):
    path = O.build(plant=plant, out=str(tmp_path / f"liboracle_plant{plant}.so"))
    bad = O.Oracle(path)
    failed = []
    for pin in P.ALL_PINS:
        try:
            pin(bad)
        except (AssertionError, FloatingPointError, ValueError, TypeError,
                __import__("numpy").linalg.LinAlgError):
            failed.append(pin.__name__)
    assert failed, f"planted mistake '{PLANTS[plant]}' passed every pin"
