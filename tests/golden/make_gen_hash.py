"""Record the generator's bit pattern for the n=64, seed=1 skew matrix (determinism pin)."""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from paper_2408_05238_amd import inputs  # noqa: E402

A = inputs.skew_gaussian(64, 1)
h = hashlib.sha256(np.asfortranarray(A).tobytes(order="F")).hexdigest()
with open(os.path.join(HERE, "skew_gaussian_n64_s1.sha256"), "w") as f:
    f.write(h + "  skew_gaussian(n=64, seed=1, stream=0), column-major float64\n")
print(h)
