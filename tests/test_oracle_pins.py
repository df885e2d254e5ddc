"""The CPU oracle against its pins (hand-worked cases, brute force, closed forms, invariants)."""
import pytest

import oracle
import synth

from . import pins


@pytest.fixture(scope="module")
def O():
    oracle.build(force=False)
    synth.build(force=False)
    return oracle.default()


@pytest.mark.parametrize("check", pins.ALL, ids=lambda f: f.__name__)
def test_pin(O, check):
    check(O)


def test_identity_document(O):
    pins.check_identity_document(O, synth)


def test_mine_composition(O):
    pins.check_mine_composition(O, synth)
