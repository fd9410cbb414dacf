"""Compute the force scale that gives the 192-atom water box a per-component force RMS of 1 eV/A.

Forces are linear in the last fitting layer, so the scale is 1 / RMS(F) of
the unscaled model.  The printed value is the ``FORCE_SCALE`` literal in
``synth/weights.py``.  Run:  python -m oracle.calibrate_force_scale
"""
import os
import sys
import tempfile

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from synth import config_system, write_model_file  # noqa: E402
from oracle.model_file import load_model  # noqa: E402
from oracle.dp import evaluate  # noqa: E402


def main():
    with tempfile.TemporaryDirectory() as d:
        path = write_model_file(os.path.join(d, "unscaled.bin"), seed=2602, force_scale=1.0)
        m = load_model(path)
    s = config_system("water192")
    out = evaluate(m, s.coords, s.types, s.box)
    rms = float(np.sqrt(np.mean(out["F"] ** 2)))
    print(repr(1.0 / rms))


if __name__ == "__main__":
    main()
