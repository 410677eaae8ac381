"""Writes hand_two_body.json: Eqs. (2), (3), (5), (6) reduced by hand.

Configuration: massive object (mass M) at rest at the origin, one star of
mass m at (r, 0, 0) with velocity (0, v, 0), no softening, G = 1.

Star (Eqs. (5), (6); no partner star j, so only the first line of Eq. (6)):
  [a_i]_BH    = (G M / r^2)(4 G M / r - v^2) x_hat          (v.x = 0)
  [a_i]_Cross = 5 G^2 m M / r^3 x_hat - 4 G m v^2 / r^2 x_hat
Massive object (Eqs. (2), (3); x_1j = x_1 - x_j = -r x_hat; the G^2 double
sums need j != k and vanish; the last line of Eq. (3) has k = j):
  [a_1]_BH    = -(G m / r^2)(5 G M / r - 2 v^2) x_hat
  [a_1]_Cross = -4 G^2 m^2 / r^3 x_hat + 4 G m^2 v^2 / (M r^2) x_hat
The stored values are these times 1/c^2 (x components; y and z vanish).
"""
import json
import os

G = 1.0
M, m, r, v, c = 1.7, 0.003, 0.8, 0.9, 12.0
lam = 1.0 / (c * c)
star = lam * ((G * M / r**2) * (4 * G * M / r - v * v) + 5 * G * G * m * M / r**3
              - 4 * G * m * v * v / r**2)
bh = lam * (-(G * m / r**2) * (5 * G * M / r - 2 * v * v) - 4 * G * G * m * m / r**3
            + 4 * G * m * m * v * v / (M * r**2))
out = dict(M=M, m=m, r=r, v=v, c=c, star_1pn_x=star, bh_1pn_x=bh,
           source="hand reduction of Sec. 2, Eqs. (2), (3), (5), (6); see make_hand_two_body.py")
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "hand_two_body.json"), "w") as f:
    json.dump(out, f, indent=1)
    f.write("\n")
