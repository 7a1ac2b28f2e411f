"""Writes blade_element_cases.json: closed-form special cases of the
blade-element force (Sec. 2.2 of the paper) with the synthetic polars,
evaluated with plain arithmetic (no solver code)."""
import json
import math
import os


def case(name, rho, wn, wt, chord, dl, twist, note):
    phi = math.degrees(math.atan2(wn, wt))
    a = phi - twist
    ar = math.radians(a)
    clip = math.radians(12.0)
    CL = 2 * math.pi * max(-clip, min(clip, ar))
    CD = 0.01 + 0.02 * ar * ar
    W = math.hypot(wn, wt)
    q = 0.5 * rho * W * W * chord * dl
    if wt == 0.0:            # frozen rotor: e_L = e_theta, e_D = e_x
        Fn, Ft = q * CD, q * CL
    elif wn == wt:           # 45 degrees: e_L = (e_x + e_t)/sqrt2, e_D = (e_x - e_t)/sqrt2
        Fn, Ft = q * (CL + CD) / math.sqrt(2), q * (CL - CD) / math.sqrt(2)
    else:                    # e_L = (wt e_x + wn e_t)/W, e_D = (wn e_x - wt e_t)/W
        Fn, Ft = q * (CL * wt + CD * wn) / W, q * (CL * wn - CD * wt) / W
    return dict(name=name, rho=rho, wn=wn, wt=wt, chord=chord, dl=dl, twist_deg=twist,
                alpha_deg=a, CL=CL, CD=CD, Fn=Fn, Ft=Ft, derivation=note)


cases = [
    case("frozen rotor, axial wind", 1.0, 0.05, 0.0, 2.7625, 0.5, 9.6875,
         "Omega = 0 and u = U e_x: W_n = U, W_t = 0, phi = 90 deg, alpha = 90 - twist = "
         "80.3125 deg (beyond stall: C_L = 2 pi * 12 deg in rad); e_L = e_theta and e_D = e_x, "
         "so Fn = q C_D, Ft = q C_L with q = rho U^2 c l / 2. Element 16 of the 16-cell-radius "
         "rotor: r = 8.25, c = 16 (0.25 - 0.15 * 8.25/16), twist = 20 (1 - 8.25/16), l = 0.5."),
    case("45 degree inflow", 1.0, 0.05, 0.05, 1.0, 1.0, 40.0,
         "W_n = W_t: phi = 45 deg, alpha = 5 deg; e_L = (e_x + e_theta)/sqrt 2, "
         "e_D = (e_x - e_theta)/sqrt 2, so Fn = q (C_L + C_D)/sqrt 2 and Ft = q (C_L - C_D)/sqrt 2."),
    case("negative angle of attack", 1.02, 0.03, 0.2, 1.5, 0.25, 15.0,
         "phi = atan(0.15) in degrees, alpha = phi - 15 deg < 0, attached (|alpha| < 12 deg)."),
]
doc = {"source": "closed-form special cases of the blade-element force equation (Sec. 2.2 of "
       "the paper): F = rho |W|^2 c l (C_L e_L + C_D e_D) / 2 with the synthetic polars "
       "C_L = 2 pi alpha (|alpha| clipped at 12 deg), C_D = 0.01 + 0.02 alpha^2 (alpha in rad). "
       "Written by make_blade_element_cases.py with plain arithmetic; the test tolerance covers "
       "the 0.1-degree polar table interpolation.", "cases": cases}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       "blade_element_cases.json"), "w") as fh:
    json.dump(doc, fh, indent=1)
