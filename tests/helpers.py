"""Shared helpers of the test-suite (no method arithmetic)."""
import numpy as np

FIELDS = ("ax", "ay", "az", "drho", "dsxx", "dsyy", "dszz", "dsxy", "dsxz", "dsyz", "rho_sum")
GROUPS = {"ax": "acc", "ay": "acc", "az": "acc", "dsxx": "dS", "dsyy": "dS", "dszz": "dS",
          "dsxy": "dS", "dsxz": "dS", "dsyz": "dS", "drho": "drho", "rho_sum": "rho_sum"}
GROUP_FLOOR = 1e-3


def split(out: dict) -> dict:
    """Per-field arrays from an output dict with acc (3, n), drho, dS (6, n), rho_sum."""
    a = np.asarray(out["acc"])
    s = np.asarray(out["dS"])
    return dict(ax=a[0], ay=a[1], az=a[2], drho=np.asarray(out["drho"]), dsxx=s[0], dsyy=s[1],
                dszz=s[2], dsxy=s[3], dsxz=s[4], dsyz=s[5], rho_sum=np.asarray(out["rho_sum"]))


def scales(ref: dict, rho=None, mu=None) -> dict:
    """Error scale of every output field: the field's own max |ref|, floored at GROUP_FLOOR
    times the max of the vector/tensor it belongs to (acceleration components, stress-rate
    components; drho against rho * |L| when the reference carries L), so that components
    that vanish by symmetry are measured against the size of their group, not against
    roundoff.  With ``mu``, a stress-rate component is measured against at least the
    Hooke term's size 2 mu max|L|, the size its rounding scales with: where the strain
    rate cancels to zero (a rigid rotation under the corrected gradient) the result is
    the rotation terms alone, far smaller than the terms that cancelled."""
    r = split(ref)
    g = {"acc": max(np.abs(r[k]).max() for k in ("ax", "ay", "az")),
         "dS": max(np.abs(r[k]).max() for k in ("dsxx", "dsyy", "dszz", "dsxy", "dsxz", "dsyz")),
         "drho": np.abs(r["drho"]).max(), "rho_sum": np.abs(r["rho_sum"]).max()}
    if "L" in ref and rho is not None:
        g["drho"] = max(g["drho"], np.abs(np.asarray(rho)).max() * np.abs(np.asarray(ref["L"])).max())
    sc = {k: max(np.abs(r[k]).max(), GROUP_FLOOR * g[GROUPS[k]]) for k in FIELDS}
    if "L" in ref and mu is not None:
        hooke = 2.0 * mu * np.abs(np.asarray(ref["L"])).max()
        for k in FIELDS:
            if GROUPS[k] == "dS":
                sc[k] = max(sc[k], hooke)
    return sc


def normwise(got: dict, ref: dict, rho=None, mu=None) -> dict:
    """max_a |got - ref| / scale for every output field (see ``scales``)."""
    gg, rr = split(got), split(ref)
    sc = scales(ref, rho, mu)
    res = {}
    for k in FIELDS:
        err = np.abs(gg[k] - rr[k]).max()
        res[k] = err / sc[k] if sc[k] > 0 else (0.0 if err == 0 else np.inf)
    return res
