"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake into a copy of the oracle's source -- a dropped term, a
wrong sign or axis, a sum over the wrong set, a wrong tie rule -- loads the copy in
place of the oracle and runs the pins of ``test_oracle_pins.py`` against it.  At
least one pin must fail for every mistake; the pins are run without the slow
main-loop check.  Nothing here touches the oracle's own file.
"""
import importlib.util
import os
import sys
import types

import pytest

import oracle
from oracle import pxst_oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "pxst_oracle.py")

# (name, text in the oracle, planted replacement)
MUTATIONS = [
    ("pixel-map refinement sign", "nu[0, p] += ox", "nu[0, p] -= ox"),
    ("pixel-map refinement axes", "nu[0, p] += ox\n                nu[1, p] += oy",
     "nu[0, p] += oy\n                nu[1, p] += ox"),
    ("translation refinement sign", "out[n, 0] = dx[n, 0] + sx + ox", "out[n, 0] = dx[n, 0] + sx - ox"),
    ("translation refinement axes", "dx[n, 0] + sx + ox\n        out[n, 1] = dx[n, 1] + sy + oy",
     "dx[n, 0] + sx + oy\n        out[n, 1] = dx[n, 1] + sy + ox"),
    ("translation variance over all pixels", "var = np.where(ok, v * v, 0.0).sum()", "var = (v * v).sum()"),
    ("translation shift sign", "ua - (dx[n, 0] + sx) - origin[0]", "ua - (dx[n, 0] - sx) - origin[0]"),
    ("error counts invalid lookups", "use = ok & (s2 > 0) & sel", "use = (s2 > 0) & sel"),
    ("reference-plane error weighted by W", "(M * eps)[sel], M[sel])", "(M * W * eps)[sel], (M * W)[sel])"),
    ("error not divided by sigma^2", "r * r / np.where(s2 > 0, s2, 1.0)", "r * r"),
    ("zero-variance rule dropped", "    E[(nv > 0) & (var == 0) & (err == 0)] = 0.0\n", ""),
    ("sigma^2 over N - 1", "return acc / frames.shape[0]", "return acc / (frames.shape[0] - 1)"),
    ("reference numerator without W", "(M * W)[sel] * I, (M * W * W)[sel]", "M[sel] * I, (M * W * W)[sel]"),
    ("reference weight M W instead of M W^2", "(M * W)[sel] * I, (M * W * W)[sel]", "(M * W)[sel] * I, (M * W)[sel]"),
    ("bilinear corner weights transposed", "(1, 0): fa * (1.0 - fb),\n            (0, 1): (1.0 - fa) * fb",
     "(1, 0): (1.0 - fa) * fb,\n            (0, 1): fa * (1.0 - fb)"),
    ("pixel-map variance about 0 instead of W", "        err += np.where(ok, r * r, 0.0)\n        v = I[n] - Wp\n",
     "        err += np.where(ok, r * r, 0.0)\n        v = I[n]\n"),
    ("translation variance about 0 instead of W", "v = I - Wp", "v = I"),
    ("pixel-map last minimum", "k = np.argmin(flat, axis=0)                       # first minimum",
     "k = flat.shape[0] - 1 - np.argmin(flat[::-1], axis=0)"),
    ("candidate centre by floor", "c = round_half_up(u_sel[:, good])\n        use",
     "c = np.floor(u_sel[:, good])\n        use"),
    ("round half up as floor(x + 1/2)", "return f + ((x - f) >= 0.5)", "return np.floor(x + 0.5)"),
    ("paraboloid cross term sign", "q4 = (x * y * E).sum() / 4.0", "q4 = -(x * y * E).sum() / 4.0"),
    ("paraboloid accepts a maximum", "if not (q3 > 0 and D > 0):", "if not (D > 0):"),
    ("paraboloid offset not clamped", "return float(np.clip(ox, -0.5, 0.5)), float(np.clip(oy, -0.5, 0.5))",
     "return float(ox), float(oy)"),
    ("masked gather ignores validity", "m = wt * (inb & valid[ia, ib])", "m = wt * inb"),
    ("splat keeps out-of-grid corners at the edge", "np.add.at(num, (ia[inb], ib[inb]), (wt * values)[inb])",
     "np.add.at(num, (ia, ib), wt * values)"),
]


def _pins():
    spec = importlib.util.spec_from_file_location("_pins_under_mutation", os.path.join(HERE, "test_oracle_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return [(n, f) for n, f in vars(mod).items()
            if n.startswith("test_") and callable(f) and n != "test_main_loop_error_decreases_on_noiseless_scan"]


def _mutant(old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    m = types.ModuleType("oracle.pxst_oracle")
    m.__file__ = SRC
    exec(compile(text.replace(old, new), SRC + " (mutated)", "exec"), m.__dict__)
    return m


def test_unmutated_oracle_passes_the_pins():
    for name, f in _pins():
        f()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new, monkeypatch):
    m = _mutant(old, new)
    monkeypatch.setitem(sys.modules, "oracle.pxst_oracle", m)
    monkeypatch.setattr(oracle, "pxst_oracle", m)
    for attr in dir(pxst_oracle):
        if not attr.startswith("__") and hasattr(oracle, attr):
            monkeypatch.setattr(oracle, attr, getattr(m, attr))
    caught = []
    for pin, f in _pins():
        try:
            f()
        except Exception:  # an assertion, or the mistake breaking the computation
            caught.append(pin)
    assert caught, f"no pin caught: {name}"
