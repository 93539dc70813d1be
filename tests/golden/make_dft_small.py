"""Writes dft_small.txt: hand-derived closed-form DFT values (textbook identities
of the definition X[k] = sum_j x[j] exp(-2 pi i j k / N); the paper names the DFT
in section III-A without a worked example).  Uses only the math module: no FFT
implementation, GPU or oracle, is involved.  Run from this folder."""
import math


def cases():
    out = []
    out.append(("n1_identity", "N=1: X[0]=x[0]", [(3.0, 2.0)], [(3.0, 2.0)]))
    out.append(("n2_butterfly", "N=2: X=[x0+x1, x0-x1]",
                [(1.0, 2.0), (3.0, -1.0)], [(4.0, 1.0), (-2.0, 3.0)]))
    out.append(("n4_ramp", "N=4, x=[1,2,3,4]: X0=10, X1=1-2i-3+4i=-2+2i, X2=1-2+3-4=-2, X3=1+2i-3-4i=-2-2i",
                [(1, 0), (2, 0), (3, 0), (4, 0)], [(10, 0), (-2, 2), (-2, 0), (-2, -2)]))
    h = math.sqrt(3) / 2
    out.append(("n3_delayed_impulse", "N=3, x=delta[j-1]: X[k]=w3^k, w3=-1/2-i*sqrt(3)/2",
                [(0, 0), (1, 0), (0, 0)], [(1, 0), (-0.5, -h), (-0.5, h)]))
    out.append(("n3_constant", "N=3, constant 1: X=[3,0,0] (sum of the cube roots of unity is 0)",
                [(1, 0)] * 3, [(3, 0), (0, 0), (0, 0)]))
    out.append(("n5_impulse", "N=5, x=delta[j]: X[k]=1 for all k", [(1, 0)] + [(0, 0)] * 4, [(1, 0)] * 5))
    out.append(("n6_alternating", "N=6, x[j]=(-1)^j = exp(-2 pi i j 3/6): X[3]=6, else 0",
                [(1, 0), (-1, 0)] * 3, [(0, 0), (0, 0), (0, 0), (6, 0), (0, 0), (0, 0)]))
    r = math.sqrt(0.5)
    w8 = [(1, 0), (r, -r), (0, -1), (-r, -r), (-1, 0), (-r, r), (0, 1), (r, r)]
    out.append(("n8_delayed_impulse", "N=8, x=delta[j-1]: X[k]=w8^k, w8=(1-i)/sqrt(2)",
                [(0, 0), (1, 0)] + [(0, 0)] * 6, w8))
    cs = [(math.cos(2 * math.pi * 2 * j / 7), math.sin(2 * math.pi * 2 * j / 7)) for j in range(7)]
    out.append(("n7_tone_f2", "N=7, x[j]=exp(+2 pi i 2j/7): X[k]=7 delta[k-2] (orthogonality of roots of unity)",
                cs, [(0, 0), (0, 0), (7, 0), (0, 0), (0, 0), (0, 0), (0, 0)]))
    return out


if __name__ == "__main__":
    with open("dft_small.txt", "w") as f:
        for name, why, x, X in cases():
            f.write(f"case {name}  # {why}\n")
            f.write(f"n {len(x)}\n")
            for a, b in x:
                f.write(f"x {a:.17g} {b:.17g}\n")
            for a, b in X:
                f.write(f"X {a:.17g} {b:.17g}\n")
            f.write("\n")
