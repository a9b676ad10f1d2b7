"""The oracle's Compton branch, its interaction-length resamples and its particle
ledger against the closed forms of the toy shower model (checks in oracle_pins.py)."""
import pytest

import oracle_pins as pins


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("E", [0.3, 0.5, 1.0, 1.02])
def test_compton_kill_fraction_and_spectrum(oracle_mod, E, precision):
    pins.compton_kill_and_spectrum(oracle_mod.lib(), E, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_compton_hand_trace(oracle_mod, precision):
    pins.compton_hand_trace(oracle_mod.lib(), precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_interaction_length_resampled_after_compton(oracle_mod, precision):
    pins.resample_after_compton(oracle_mod.lib(), precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_interaction_length_resampled_after_brem(oracle_mod, precision):
    pins.resample_after_brem(oracle_mod.lib(), precision)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_particle_ledger_and_charge(oracle_mod, precision, scheme):
    pins.ledger_mixed_shower(oracle_mod.lib(), precision, scheme)
