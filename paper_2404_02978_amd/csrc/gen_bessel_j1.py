"""Writes the coefficients of the device's J1 (qrfs_device.hpp, j1x_pi).

J1(x)/x is needed for the circular-aperture filter of Eq. 7,
F = 2 (D^2 J1(x_D)/x_D - d^2 J1(x_d)/x_d) / (D^2 - d^2), x = pi D f.
  x < 8:  J1(x)/x = sum_n a_n (x^2 - 32)^n, n <= 16, a least-squares fit at
          Chebyshev nodes of z = x^2 in [0, 64] of the entire function
          J1(sqrt z)/sqrt z (its power series, DLMF 10.2.2, is the origin);
          centring on z = 32 keeps the Horner sum free of cancellation.
  x >= 8: Hankel's form (DLMF 10.17.3) J1(x) = sqrt(2/(pi x))
          (P(x) cos chi - Q(x) sin chi), chi = x - 3 pi/4, with P and
          x Q / 8 fitted as polynomials of degree 8 in w = (8/x)^2 in (0, 1],
          from P = sqrt(pi x/2) (J1 cos chi + Y1 sin chi) and
          Q = sqrt(pi x/2) (Y1 cos chi - J1 sin chi).
For the FP32-class weights and basis values (j1x_pi_f32) the same two forms
with fewer terms: the x < 8 polynomial of degree 10 (evaluated in binary64,
fit error 1.2e-10) and P, x Q / 8 of degree 3 (evaluated in binary32, fit
error 6e-11 in J1(x)/x).
The reference values come from mpmath at 60 digits.  Run:
    python gen_bessel_j1.py      (prints the C++ constant tables)
"""
import mpmath as mp

mp.mp.dps = 60


def lsq(nodes, vals, deg, var):
    A = mp.matrix([[var(t) ** j for j in range(deg + 1)] for t in nodes])
    return mp.lu_solve(A.T * A, A.T * mp.matrix(vals))


def small(deg=16, n=24):
    zs = [32 * (1 + mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n)) for k in range(n)]
    vals = [mp.besselj(1, mp.sqrt(z)) / mp.sqrt(z) for z in zs]
    c = lsq(zs, vals, deg, lambda z: (z - 32) / 32)  # fitted in [-1, 1]
    return [c[j] / mp.mpf(32) ** j for j in range(deg + 1)]


def large(deg=8, n=20):
    ws = [(1 + mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n)) / 2 for k in range(n)]
    P, q = [], []
    for w in ws:
        x = 8 / mp.sqrt(w)
        chi = x - 3 * mp.pi / 4
        j, y = mp.besselj(1, x), mp.bessely(1, x)
        s = mp.sqrt(mp.pi * x / 2)
        P.append(s * (j * mp.cos(chi) + y * mp.sin(chi)))
        q.append(s * (y * mp.cos(chi) - j * mp.sin(chi)) * x / 8)
    return lsq(ws, P, deg, lambda w: w), lsq(ws, q, deg, lambda w: w)


def table(name, c, ctype="double", digits=20):
    body = ",\n    ".join(mp.nstr(v, digits, min_fixed=-1, max_fixed=-1) +
                          ("f" if ctype == "float" else "") for v in c)
    return f"constexpr {ctype} {name}[{len(c)}] = {{\n    {body}}};"


if __name__ == "__main__":
    a = small()
    p, q = large()
    print(table("kJ1Small", a))
    print(table("kJ1P", p))
    print(table("kJ1Q", q))
    print(table("kJ1Small10", small(deg=10, n=18)))
    p3, q3 = large(deg=3, n=11)
    print(table("kJ1P3", p3, "float", 9))
    print(table("kJ1Q3", q3, "float", 9))
