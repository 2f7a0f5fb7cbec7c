"""Writes wendland_eq8.json: eps*phi(u) of Eq. (8) at rational u, in exact
rational arithmetic (Python fractions), independent of every compiled path."""
import json
import os
from fractions import Fraction as F

pts = [F(0), F(1, 4), F(1, 2), F(3, 4), F(1)]
vals = []
for u in pts:
    v = u * u * ((u * (u * (3 * u - 15) + 28) - 21) * u * u + 7) - 3
    vals.append([float(u), float(v)])
out = {"source": "Eq. (8) of the paper (Sec. 2.3): phi(r) = (1/eps) (u^2 ((u (u (3u - 15) + 28) - 21) u^2 + 7) - 3), u = r/eps < 1; values of eps*phi at rational u, evaluated exactly with Python fractions by tests/golden/make_wendland_golden.py",
       "eps": 0.25, "phi_times_eps": vals}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "wendland_eq8.json"), "w") as f:
    json.dump(out, f, indent=1)
