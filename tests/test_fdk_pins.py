"""The FDK pre-processing oracle against its pins, and planted mistakes against the pins (CPU only)."""
import importlib.util
import os

import pytest

import fdk_pins as pins
from oracle import fdk

SRC = fdk.__file__

MUTANTS = {
    "tau_not_magnified": ("return pitch * sid / sdd", "return pitch"),
    "no_tau_scale": ("return tau * (x @ ramp_matrix(x.shape[-1], tau))", "return x @ ramp_matrix(x.shape[-1], tau)"),
    "ramp_sign": ("h[odd] = -1.0 / (np.pi", "h[odd] = 1.0 / (np.pi"),
    "even_taps_nonzero": ("odd = (np.abs(n) % 2) == 1", "odd = n != 0"),
    "centre_tap": ("h[n == 0] = 1.0 / (4.0 * tau * tau)", "h[n == 0] = 1.0 / (2.0 * tau * tau)"),
    "missing_pi": ("-1.0 / (np.pi * np.pi * nf * nf * tau * tau)", "-1.0 / (nf * nf * tau * tau)"),
    "orientation": ("ramp_taps(m[None, :] - m[:, None], tau)", "ramp_taps(m[None, :] + m[:, None], tau)"),
    "weight_no_v": ("sdd * sdd + u[None, :] ** 2 + v[:, None] ** 2", "sdd * sdd + u[None, :] ** 2 + 0.0 * v[:, None]"),
    "weight_inverted": ("return sdd / np.sqrt(", "return (1.0 / sdd) * np.sqrt("),
    "pixel_corner": ("u = (np.arange(W, dtype=np.float64) - (W - 1) / 2.0) * pitch",
                     "u = (np.arange(W, dtype=np.float64) - W / 2.0) * pitch"),
    "weight_not_applied": ("p * cosine_weights(W, H, pitch, sdd)[None], tau)", "p, tau)"),
    "rows_wrong_weight_row": ("* c[j] for k, j in rows", "* c[0] for k, j in rows"),
}


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_fdk_oracle_pin(pin):
    pin(fdk)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_fdk_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / f"fdk_{name}.py"
    path.write_text(text.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"fdk_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(mod)
        except AssertionError as e:
            failed.append(f"{pin.__name__}: {str(e)[:80]}")
    assert failed, f"no pin catches mutant {name}"
