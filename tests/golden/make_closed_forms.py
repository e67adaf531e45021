"""Write closed_forms.json: values of formulas printed in arXiv:1708.03912,
evaluated in 40-digit arithmetic (mpmath).  No oracle or library code runs
here; each entry names the passage it evaluates.

    python tests/golden/make_closed_forms.py
"""
import json
import os

import mpmath as mp

mp.mp.dps = 40


def C(d, s):
    # Sec. 2: C(d,s) = 2^{2s} s Gamma(s+d/2) / (pi^{d/2} Gamma(1-s))
    return mp.power(2, 2 * s) * s * mp.gamma(s + mp.mpf(d) / 2) / (mp.power(mp.pi, mp.mpf(d) / 2) * mp.gamma(1 - s))


def ball_c(d, s):
    # Sec. 7, n = l = 0: f_{0,0} = 2^{2s} Gamma(1+s)^2 binom(s+d/2-1, s) ... gives
    # u = (1-|x|^2)^s; dividing by f_{0,0} yields the solution for f = 1.
    # 1D: f_{0,0}^{1D} = 2^{2s} Gamma(1+s)^2 binom(s-1/2, s) binom(s, s)
    # 2D: f_{0,0}^{2D} = 2^{2s} Gamma(1+s)^2 binom(s, s) binom(s, s)
    binom = lambda x, y: mp.gamma(x + 1) / (mp.gamma(y + 1) * mp.gamma(x - y + 1))
    if d == 1:
        f00 = mp.power(2, 2 * s) * mp.gamma(1 + s) ** 2 * binom(s - mp.mpf(1) / 2, s) * binom(s, s)
    else:
        f00 = mp.power(2, 2 * s) * mp.gamma(1 + s) ** 2 * binom(s, s) * binom(s, s)
    return 1 / f00


def ball_fu(d, s):
    # (f,u) = int_{B} c (1-|x|^2)^s dx
    c = ball_c(d, s)
    if d == 1:
        return c * mp.quad(lambda x: (1 - x * x) ** s, [-1, 1])
    return c * 2 * mp.pi * mp.quad(lambda r: (1 - r * r) ** s * r, [0, 1])


def sign_fu(s):
    # Sec. 7.1, f = sign(x) on (-1,1): (f,u) = 2^{1-2s} / ((2s+1) Gamma(1+s)^2)
    return mp.power(2, 1 - 2 * s) / ((2 * s + 1) * mp.gamma(1 + s) ** 2)


out = {"_source": "arXiv:1708.03912; values of the printed formulas (mpmath, 40 digits)", "entries": []}
for d in (1, 2):
    for s in ("0.25", "0.5", "0.75"):
        sv = mp.mpf(s)
        out["entries"].append({"quantity": "C(d,s)", "d": d, "s": float(sv), "cite": "Sec. 2, normalisation constant",
                               "value": mp.nstr(C(d, sv), 30)})
        out["entries"].append({"quantity": "ball_c", "d": d, "s": float(sv),
                               "cite": "Sec. 7, closed-form solutions with n = 0 (and l = 0)",
                               "value": mp.nstr(ball_c(d, sv), 30)})
        out["entries"].append({"quantity": "ball_fu", "d": d, "s": float(sv),
                               "cite": "Sec. 7, (f,u) for f = 1 on the unit ball",
                               "value": mp.nstr(ball_fu(d, sv), 30)})
for s in ("0.25", "0.75"):
    out["entries"].append({"quantity": "sign_fu", "d": 1, "s": float(s), "cite": "Sec. 7.1, discontinuous right-hand side",
                           "value": mp.nstr(sign_fu(mp.mpf(s)), 30)})
# Sec. 3 example: on the unit disk f = 2^{2s} Gamma(1+s)^2 gives u = (1-|x|^2)^s
for s in ("0.25", "0.75"):
    sv = mp.mpf(s)
    out["entries"].append({"quantity": "disk_example_f", "d": 2, "s": float(sv),
                           "cite": "Sec. 3, example after the regularity theorem",
                           "value": mp.nstr(mp.power(2, 2 * sv) * mp.gamma(1 + sv) ** 2, 30)})
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json"), "w") as f:
    json.dump(out, f, indent=1)
print("wrote", len(out["entries"]), "entries")
