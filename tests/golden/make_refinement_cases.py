"""Writes refinement_cases.json: tiny one-outer-step refinement cases whose
results follow by hand.

Each case is one outer step of mixed-precision iterative refinement with
Jacobi inner sweeps on the correction equation (the refinement form of the
Jacobi3D workload, paper section 4.3, with the storage readings: binary64
residual r = (b + s) - 6u, r_lo = r rounded to binary32 and, for bfloat16
storage, from there to bfloat16, round to nearest even; inner sweeps from
d = 0 with zero ghosts, d' = lo(((s(d) + r_lo) / 6)) with binary32 sums
taken in the order x-, x+, y-, y+, z-, z+ and a binary32 division; update
u + d in binary64).

Every expected value is stated by hand in the case (with its derivation)
and is also recomputed here in exact rational arithmetic with an explicit
round-to-nearest-even to each format; the script refuses to write a case
where the two disagree.  No oracle or GPU code is called.
Run: python tests/golden/make_refinement_cases.py
"""
import json
import os
from fractions import Fraction as Fr

# ------------------------------------------------ exact rounding ----------

FORMATS = {"f64": (53, -1022, 1023), "f32": (24, -126, 127), "bf16": (8, -126, 127)}


def rne(x, fmt):
    """x (a Fraction) rounded to nearest, ties to even, in a binary format
    with p significand bits (implicit bit included), subnormals below
    2^emin, overflow to infinity."""
    p, emin, emax = FORMATS[fmt]
    x = Fr(x)
    if x == 0:
        return Fr(0)
    sgn = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fr(2) ** e > a:
        e -= 1
    while Fr(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    ulp = Fr(2) ** (e - p + 1)
    q = a / ulp
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and n % 2 == 1):
        n += 1
    r = n * ulp
    if r >= Fr(2) ** (emax + 1):
        raise OverflowError("case overflows")
    return sgn * r


def lo(x, storage):
    """binary32 value x rounded to the storage format (bfloat16 via binary32)."""
    return rne(x, "bf16") if storage == "bf16" else x


# -------------------------------------------- one outer step, exactly ------

def outer_step(n, u, b, storage, m):
    """u, b: dicts (x, y, z) -> Fraction over the padded grid (missing = 0)."""
    nx, ny, nz = n
    cells = [(x, y, z) for z in range(1, nz + 1) for y in range(1, ny + 1) for x in range(1, nx + 1)]
    nbrs = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))

    def at(a, c):
        return a.get(c, Fr(0))

    rlo = {}
    for c in cells:
        s = Fr(0)
        for k, (dx, dy, dz) in enumerate(nbrs):
            v = at(u, (c[0] + dx, c[1] + dy, c[2] + dz))
            s = v if k == 0 else rne(s + v, "f64")
        r = rne(rne(at(b, c) + s, "f64") - rne(6 * at(u, c), "f64"), "f64")
        rlo[c] = lo(rne(r, "f32"), storage)
    d = {}
    for _ in range(m):
        e = {}
        for c in cells:
            s = Fr(0)
            for k, (dx, dy, dz) in enumerate(nbrs):
                v = at(d, (c[0] + dx, c[1] + dy, c[2] + dz))   # ghosts of d are 0
                s = v if k == 0 else rne(s + v, "f32")
            e[c] = lo(rne(rne(s + rlo[c], "f32") / 6, "f32"), storage)
        d = e
    return [rne(at(u, c) + d[c], "f64") for c in cells]


# ------------------------------------------------------------- cases -------

def padded_list(n, vals):
    """Flat padded (nz+2, ny+2, nx+2) list, x fastest, from {(x, y, z): value}."""
    nx, ny, nz = n
    return [float(vals.get((x, y, z), Fr(0))) for z in range(nz + 2) for y in range(ny + 2)
            for x in range(nx + 2)]


cases = []


def add(name, n, storage, m, b, expected, derivation, u0=None):
    u0 = u0 or {}
    got = outer_step(n, u0, b, storage, m)
    exp = [Fr(v) for v in expected]
    if got != exp:
        raise SystemExit("case %s: hand value %s, exact arithmetic %s"
                         % (name, [float(v) for v in exp], [float(v) for v in got]))
    for v in list(b.values()) + list(u0.values()):
        assert Fr(float(v)) == v, "input of %s not a binary64 value" % name
    cases.append(dict(name=name, n=list(n), storage=storage, inner=m,
                      u0=padded_list(n, u0), b=padded_list(n, b),
                      expected_interior=[float(v) for v in exp],
                      expected_hex=[float(v).hex() for v in exp], derivation=derivation))


P = lambda k: Fr(2) ** k   # noqa: E731

add("bf16_residual_through_binary32", (1, 1, 1), "bf16", 1,
    {(1, 1, 1): 1 + P(-8) + P(-30)},
    [Fr(171, 1024)],
    "g = 0, u0 = 0, so r = b = 1 + 2^-8 + 2^-30.  To binary32: 2^-30 is below half an ulp "
    "(2^-24), r32 = 1 + 2^-8.  To bfloat16: 1 + 2^-8 is the tie between 1 and 1 + 2^-7, even "
    "gives r_lo = 1.  One cell with zero ghosts: d = lo(1/6); binary32 1/6 = 0x3E2AAAAB, whose "
    "bfloat16 neighbours are 170/1024 and 171/1024 with 1/6 * 1024 = 170.67, so d = 171/1024.  "
    "Rounding r straight from binary64 to bfloat16 would give 1 + 2^-7 (above the tie) and "
    "d = lo((1 + 2^-7)/6) = 43/256.")

add("bf16_residual_rounded_to_storage", (1, 1, 1), "bf16", 3,
    {(1, 1, 1): 1 + P(-7) + 3 * P(-10) + P(-20)},
    [Fr(43, 256)],
    "r = b = 1 + 2^-7 + 3*2^-10 + 2^-20 is a binary32 value; to bfloat16 (ulp 2^-7, the part "
    "above 1 + 2^-7 is below half an ulp): r_lo = 1 + 2^-7.  Every inner sweep of the single "
    "cell gives d = lo(r_lo/6) = lo(129/768) = lo(43/256) = 43/256 exactly.  Keeping r_lo at "
    "binary32 would give r/6 just above 172.5/1024, i.e. d = 173/1024.")

add("f32_residual_rounded_to_storage", (1, 1, 1), "f32", 2,
    {(1, 1, 1): 1 + P(-24) + P(-28)},
    [Fr(int("2AAAAC", 16) | 0x800000, 2 ** 26)],
    "r = b = 1 + 2^-24 + 2^-28 rounds to binary32 r_lo = 1 + 2^-23 (above half an ulp).  "
    "1/6 lies 2/3 of an ulp (2^-26) above the binary32 value 0x3E2AAAAA; (1 + 2^-23)/6 adds "
    "4/3 ulp, exactly 2 ulps above it, so d = 0x3E2AAAAC = 0xAAAAAC * 2^-26 (as 0x2AAAAC with the "
    "implicit bit).  Dividing the unrounded binary64 r would land 1.375 ulps above, i.e. "
    "0x3E2AAAAB.")

add("bf16_correction_rounded_between_sweeps", (2, 1, 1), "bf16", 2,
    {(1, 1, 1): Fr(1, 8), (2, 1, 1): Fr(5)},
    [Fr(163, 1024), Fr(214, 256)],
    "Cells A (x = 1, r = 1/8) and B (x = 2, r = 5).  Sweep 1 (d = 0): A = lo(1/48) = 171/8192 "
    "(1/48 * 8192 = 170.67), B = lo(5/6) = 213/256 (5/6 * 256 = 213.33).  Sweep 2: A = "
    "lo((213/256 + 1/8)/6) = lo(245/1536) = 163/1024 (163.33); B = lo((171/8192 + 5)/6) = "
    "214/256 (214.22).  With B's first value kept at binary32 (5/6) instead of bfloat16, A "
    "would be lo(0.8333 + 0.125)/6 = lo(0.15972) = 164/1024.")

add("bf16_binary32_neighbour_sum", (3, 2, 1), "bf16", 2,
    {(1, 2, 1): Fr(27), (3, 2, 1): Fr(9, 128), (2, 1, 1): 3 * P(-21)},
    [Fr(3, 4), P(-22), P(-9), Fr(9, 2), Fr(3, 4), Fr(3, 256)],
    "Sweep 1 gives r/6 exactly: 4.5 at (1,2), 3/256 at (3,2), 2^-22 at (2,1), 0 elsewhere.  "
    "Sweep 2 at C = (2,2): s = (4.5 + 3/256) + 2^-22 in binary32; 4.51171875 is a multiple of "
    "2^-20 and 2^-22 is exactly half an ulp (2^-21), so the tie keeps s = 4.51171875; "
    "s/6 = 0.751953125, the bfloat16 tie between 0.75 and 0.75390625, even gives 0.75.  A "
    "binary64 neighbour sum keeps the 2^-22, s/6 becomes 0.751953125 + 2^-22/6, which rounds "
    "up to 0.751953125 + 2^-24 in binary32 and to 0.75390625 in bfloat16.  (1,1): "
    "(2^-22 + 4.5) ties back to 4.5, 4.5/6 = 0.75; (3,1): (2^-22 + 3/256)/6 rounds to 2^-9; "
    "the others keep r/6.  Order z, y, x: (1,1), (2,1), (3,1), (1,2), (2,2), (3,2).")

add("f32_binary32_neighbour_sum", (3, 2, 1), "f32", 2,
    {(1, 2, 1): Fr(27), (3, 2, 1): 3 * P(-20), (2, 1, 1): 3 * P(-22)},
    [Fr(3, 4), P(-23), rne((P(-21) + P(-23)) / 6, "f32"),
     Fr(9, 2), Fr(3, 4) + P(-24), P(-21)],
    "Sweep 1 gives r/6 exactly: 4.5 at (1,2), 2^-21 at (3,2), 2^-23 at (2,1), 0 elsewhere.  "
    "Sweep 2 at C = (2,2): s = (4.5 + 2^-21) + 2^-23 in binary32; the first sum is exact, "
    "2^-23 is a quarter ulp (2^-21) and is lost; s/6 = 0.75 + (4/3) 2^-24 rounds to "
    "0.75 + 2^-24.  A binary64 neighbour sum keeps the 2^-23: 0.75 + (5/3) 2^-24 rounds to "
    "0.75 + 2^-23.  (1,1): s = (2^-23 + 0) + 4.5 = 4.5 (a quarter ulp lost), 0.75; (3,1): "
    "s = 2^-23 + 2^-21 exactly, then RN32(s/6); the others keep r/6.  Order z, y, x: (1,1), "
    "(2,1), (3,1), (1,2), (2,2), (3,2).")

add("f32_update_in_binary64", (1, 1, 1), "f32", 1,
    {},
    [Fr(0.1) + rne(rne(rne(-rne(6 * Fr(0.1), "f64"), "f32"), "f32") / 6, "f32")],
    "u0 = 0.1 (binary64), g = 0, b = 0: r = -RN64(6 * 0.1) = -0.6000000000000001; r_lo = "
    "binary32(-0.6) = -0.60000002384; d = RN32(r_lo / 6) = -0.10000000149 (binary32 -0.1); "
    "u = 0.1 + d in binary64 = -1.49e-9 exactly (Sterbenz), not 0 as a binary32 update gives.",
    u0={(1, 1, 1): Fr(0.1)})

out = dict(source="One outer step of iterative refinement with Jacobi inner sweeps on the "
                  "correction equation (Jacobi3D workload, paper section 4.3); storage readings: "
                  "r rounded to binary32, bfloat16 through binary32, round to nearest even; "
                  "binary32 neighbour sums in x-, x+, y-, y+, z-, z+ order; binary64 update",
           layout="padded (nz+2, ny+2, nx+2), x fastest; Dirichlet shell 0; expected_interior "
                  "= u after one outer step with `inner` inner sweeps, in z, y, x order",
           cases=cases)
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "refinement_cases.json"), "w") as f:
    json.dump(out, f, indent=1)
print("wrote %d cases" % len(cases))
