"""Writes hand_cases.json: tiny Jacobi cases whose results follow by hand.

No oracle or GPU code is called; every expected value is a closed form
stated in its case's "derivation" (sums of small integers are exact, so
each value is the correctly rounded quotient of two integers).
Run: python tests/golden/make_hand_cases.py
"""
import json
import os


def padded(nx, ny, nz, fill):
    return [[[fill for _ in range(nx + 2)] for _ in range(ny + 2)] for _ in range(nz + 2)]


def flat(a):
    return [v for plane in a for row in plane for v in row]


cases = []

# 1^3: the single cell averages its six face neighbours (+ b/6).
u = padded(1, 1, 1, 100.0)          # edge/corner shell cells are never read
u[1][1][1] = 0.0
u[1][1][0], u[1][1][2] = 1.0, 2.0    # x-, x+
u[1][0][1], u[1][2][1] = 3.0, 4.0    # y-, y+
u[0][1][1], u[2][1][1] = 5.0, 9.0    # z-, z+
cases.append(dict(name="one_cell", n=[1, 1, 1], u0=flat(u), b=None, sweeps=1,
                  expected_interior=[4.0],
                  derivation="(1+2+3+4+5+9)/6 = 24/6 = 4; edge and corner shell cells (100) unused"))
b = padded(1, 1, 1, 0.0)
b[1][1][1] = 6.0
cases.append(dict(name="one_cell_source", n=[1, 1, 1], u0=flat(u), b=flat(b), sweeps=3,
                  expected_interior=[5.0], residual_u0=30.0,
                  derivation="(24 + b)/6 = 30/6 = 5, a fixed point after one sweep; "
                             "r(u0) = (b + s) - 6*0 = 30"))

# 2 x 1 x 1: A = (6 + B)/6, B = (A + 12)/6 from zero.
u = padded(2, 1, 1, 0.0)
u[1][1][0] = 6.0
u[1][1][3] = 12.0
cases.append(dict(name="two_cells_two_sweeps", n=[2, 1, 1], u0=flat(u), b=None, sweeps=2,
                  expected_interior=[8.0 / 6.0, 13.0 / 6.0],
                  derivation="sweep 1: A=6/6=1, B=12/6=2; sweep 2: A=(6+2)/6=RN(4/3), B=(1+12)/6=RN(13/6)"))

# 3^3, shell 1, interior 0: one sweep gives (number of shell neighbours)/6.
u = padded(3, 3, 3, 1.0)
for z in range(1, 4):
    for y in range(1, 4):
        for x in range(1, 4):
            u[z][y][x] = 0.0
exp = []
for z in range(1, 4):
    for y in range(1, 4):
        for x in range(1, 4):
            k = sum(1 for c in (x, y, z) for _ in (0,) if c == 1) + sum(1 for c in (x, y, z) if c == 3)
            exp.append(k / 6.0)
cases.append(dict(name="cube3_shell_one", n=[3, 3, 3], u0=flat(u), b=None, sweeps=1,
                  expected_interior=exp,
                  derivation="a cell with k coordinates on {1,3} has k shell neighbours: corners 3/6, "
                             "edges 2/6, face centres 1/6, centre 0"))

out = dict(source="Jacobi3D 7-point update, paper section 4.3; hand-derived closed forms",
           layout="padded (nz+2, ny+2, nx+2), x fastest; expected_interior in z, y, x order",
           cases=cases)
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "hand_cases.json"), "w") as f:
    json.dump(out, f, indent=1)
