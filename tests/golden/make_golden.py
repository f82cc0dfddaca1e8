"""Writes the closed-form fixtures of this folder (no oracle, no GPU code).

vmf_rows.txt: row masses of a vMF lobe about +z on an H-row equal-area map.
For a vMF lobe of concentration k about +z the cosine z = cos(theta) has the
CDF F(z) = (exp(k z) - exp(-k)) / (exp(k) - exp(-k)) on [-1, 1] (Wood 1994),
so row b of an H-row map, z in [-1 + 2b/H, -1 + 2(b+1)/H), carries mass
F(top) - F(bottom).  Written with expm1 to keep the small masses exact.
"""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def row_masses(k, H):
    # F(z) = (exp(k(z+1)) - 1) / (exp(2k) - 1) after multiplying by exp(k)
    den = math.expm1(2.0 * k)
    out = []
    for b in range(H):
        z0 = -1.0 + 2.0 * b / H
        z1 = -1.0 + 2.0 * (b + 1) / H
        # mass = (e^{k(z1+1)} - e^{k(z0+1)}) / (e^{2k} - 1)
        m = math.exp(k * (z0 + 1.0)) * math.expm1(k * (z1 - z0)) / den
        out.append(m)
    return out


def main():
    with open(os.path.join(HERE, "vmf_rows.txt"), "w") as f:
        f.write("# vMF lobe about +z: kappa H row mass (closed form, see make_golden.py)\n")
        for k in (20.0, 200.0):
            for H in (32, 64):
                for b, m in enumerate(row_masses(k, H)):
                    f.write(f"{k:g} {H} {b} {m:.17g}\n")


if __name__ == "__main__":
    main()
