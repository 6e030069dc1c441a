"""Writes adam_three_steps.json: three steps of the Adam recursions of
Kingma & Ba (2015, Alg. 1, with bias correction) evaluated in 50-digit
decimal arithmetic, as the paper's Alg. 1 uses them (the registration shift
is the gradient g_t; the position moves by +lr mhat / (sqrt(vhat) + eps),
Eq. 8-9).  Independent of the oracle and of the HIP library: it imports
neither.  Run from the repository root:
    python tests/golden/make_adam_three_steps.py
"""
import json
import os
from decimal import Decimal, getcontext

getcontext().prec = 50
LR, B1, B2, EPS = Decimal("0.5"), Decimal("0.9"), Decimal("0.999"), Decimal("1e-8")
G = [Decimal("1.0"), Decimal("-2.0"), Decimal("0.5")]


def steps():
    m = v = x = Decimal(0)
    out = {"m": [], "v": [], "x": []}
    for t, g in enumerate(G, start=1):
        m = B1 * m + (1 - B1) * g
        v = B2 * v + (1 - B2) * g * g
        mhat = m / (1 - B1 ** t)
        vhat = v / (1 - B2 ** t)
        x = x + LR * mhat / (vhat.sqrt() + EPS)
        out["m"].append(m)
        out["v"].append(v)
        out["x"].append(x)
    return out


def main():
    r = steps()
    doc = {
        "source": "Adam recursions of Kingma & Ba (2015), Alg. 1, with bias correction; the paper's Alg. 1 "
                  "feeds the registration shift in as the gradient g_t and moves the position by "
                  "+lr*mhat/(sqrt(vhat)+eps) (Eq. 8-9). Written by tests/golden/make_adam_three_steps.py "
                  "(50-digit decimal arithmetic).",
        "lr": float(LR), "b1": float(B1), "b2": float(B2), "eps": float(EPS),
        "g": [float(g) for g in G],
        "m": [float(v) for v in r["m"]],
        "v": [float(v) for v in r["v"]],
        "x": [float(v) for v in r["x"]],
        "x_50_digits": [str(v) for v in r["x"]],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adam_three_steps.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
