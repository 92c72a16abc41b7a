"""Writes advection_eq10.json: the paper's closed-form advection solution
(Eq. 10, simple advection test of Sec. 4.1.1) evaluated at t = 10, plus the
convergence orders the paper reports for that test.  Uses only the formula."""
import json
import math
import os

s3 = math.sqrt(3.0)
t = 10.0
xp = 2 / math.pi * math.atan(0.5 * (s3 * math.tan(math.pi * (s3 + 9 * t) / (6 * s3)) - 1))
out = {
    "source": "Eq. 10 (inverse of Eq. 9), simple advection test, Sec. 4.1.1: x'(t) for dx'/dt = 2 + sin(pi x'), x'(0) = 0, periodic on [-1, 1]",
    "t": t,
    "x_prime": round(xp, 12),
    "integration_constant_eq9": -1 / (3 * s3),
    "expected_order_rk2": 2,
    "expected_order_rk3": 3,
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "advection_eq10.json"), "w") as fh:
    json.dump(out, fh, indent=1)
    fh.write("\n")
print(out)
