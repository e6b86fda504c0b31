"""Shared comparison helpers of the GPU parity tests (HIP path against the FP64 oracle)."""
import math

import numpy as np

I6 = np.array([1, 1, 1, 0, 0, 0.0])[:, None]


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def grid_shape(wl):
    g = wl["grid"]
    return g["nx"], g["ny"], g["nz"]


def _phi(rho):
    return (rho[0] - rho[1]) / (rho[0] + rho[1]) if rho.shape[0] == 2 else np.ones(rho.shape[1])


def _minors(C):
    c0, c1, c2, c3, c4, c5 = C
    m2 = c0 * c1 - c3 * c3
    m3 = c0 * (c1 * c2 - c5 * c5) - c3 * (c3 * c2 - c5 * c4) + c4 * (c3 * c5 - c1 * c4)
    return np.minimum(c0, np.minimum(m2, m3))


def diag_from_fields(fields, shape, params):
    """The diagnostics record evaluated directly from host fields (rho, u, C) in FP64 with
    numpy: conservation sums, the droplet's weight w = max(phi, 0), centroid, central second
    moments, D = (a - b)/(a + b) and theta from the x-y block (Sec. 4.1 definitions), the
    FENE-P bounds and the polymer-phase mean of tr C - 3 weighted by the feedback
    modulation."""
    rho, u, C = fields
    nx, ny, nz = shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X, Y, Z = X.ravel().astype(float), Y.ravel().astype(float), Z.ravel().astype(float)
    rt = rho.sum(0)
    phi = _phi(rho)
    w = np.maximum(phi, 0.0)
    W = w.sum()
    d = {"mass_A": rho[0].sum(), "mass_B": rho[1].sum() if rho.shape[0] == 2 else 0.0,
         "mom_x": (rt * u[0]).sum(), "mom_y": (rt * u[1]).sum(), "mom_z": (rt * u[2]).sum(), "W": W}
    if W > 0:
        c = [(w * X).sum() / W, (w * Y).sum() / W, (w * Z).sum() / W]
        dx, dy, dz = X - c[0], Y - c[1], Z - c[2]
        M = [(w * a * b).sum() / W for a, b in ((dx, dx), (dy, dy), (dz, dz), (dx, dy), (dx, dz), (dy, dz))]
        d.update(xc=c[0], yc=c[1], zc=c[2], Mxx=M[0], Myy=M[1], Mzz=M[2], Mxy=M[3], Mxz=M[4], Myz=M[5])
        tr, df = M[0] + M[1], M[0] - M[1]
        rad = math.sqrt(0.25 * df * df + M[3] * M[3])
        l1, l2 = 0.5 * tr + rad, max(0.5 * tr - rad, 0.0)
        a, b = math.sqrt(l1), math.sqrt(l2)
        d["D"] = (a - b) / (a + b) if a + b > 0 else 0.0
        d["theta_deg"] = 0.5 * math.degrees(math.atan2(2 * M[3], df)) if rad > 0 else 0.0
        d["_lam_gap"] = l1 - l2
        d["_rmax"] = float(np.sqrt(dx * dx + dy * dy + dz * dz)[w > 0].max())
    d["min_L2_minus_trC"] = (params["L2"] - C[:3].sum(0)).min()
    d["min_minor"] = _minors(C).min()
    d["max_u"] = np.sqrt((u * u).sum(0)).max()
    ph = params.get("polymer_phase", "none")
    if ph == "all":
        m = np.ones_like(phi)
    elif ph in ("A", "B"):
        t = np.tanh(phi / params.get("delta", 0.1))
        m = 0.5 * (1 + t) if ph == "A" else 0.5 * (1 - t)
    else:
        m = np.zeros_like(phi)
    d["poly_trace_excess"] = (m * (C[:3].sum(0) - 3)).sum() / m.sum() if m.sum() > 0 else 0.0
    d["_w"] = w
    d["_m"] = m
    return d


_SUM_KEYS = ("mass_A", "mass_B", "mom_x", "mom_y", "mom_z", "W")


def _close(a, b, scale, rtol):
    return abs(a - b) <= rtol * max(abs(b), scale)


def check_diag(dg, do, tag, g, r, shape, params):
    """Every field of the GPU diagnostics record against the oracle's.

    1. Each record equals the definitions evaluated with numpy over its own fields to FP64
       rounding (relative 1e-9 for the sums, which only change order; 1e-12 for extrema):
       the GPU's deterministic reductions and the oracle's serial sums both compute what
       they define.
    2. The records differ by no more than the field differences allow: mass, momentum, W
       and the extrema are 1-Lipschitz in the fields they sum or bound (|max|a| - max|b|| <=
       max|a - b| and so on); the centroid and the central moments are moments of w about
       their own centre, whose first-order change is bounded by sum|dw| times the largest
       lever arm over W; theta moves by at most the moment change over the gap of the
       x-y block's eigenvalues (Davis-Kahan), D by its first-order change."""
    ng = diag_from_fields(g, shape, params)
    no = diag_from_fields(r, shape, params)
    N = g[0].shape[1]
    mscale = max(no["mass_A"], 1e-300)
    for rec, ref, who in ((dg, ng, "gpu"), (do, no, "oracle")):
        for k in _SUM_KEYS:
            sc = mscale * (max(ref["max_u"], 1e-12) if k.startswith("mom") else 1.0)
            assert _close(rec[k], ref[k], sc, 1e-9), (tag, who, k, rec[k], ref[k])
        for k in ("min_L2_minus_trC", "min_minor", "max_u"):
            assert _close(rec[k], ref[k], 1.0, 1e-12), (tag, who, k, rec[k], ref[k])
        if ref["W"] > 0:
            ext = ref["Mxx"] + ref["Myy"] + ref["Mzz"]
            for k in ("xc", "yc", "zc"):
                assert _close(rec[k], ref[k], max(shape), 1e-10), (tag, who, k, rec[k], ref[k])
            for k in ("Mxx", "Myy", "Mzz", "Mxy", "Mxz", "Myz"):
                assert _close(rec[k], ref[k], ext, 1e-9), (tag, who, k, rec[k], ref[k])
            assert abs(rec["D"] - ref["D"]) < 1e-9, (tag, who, "D", rec["D"], ref["D"])
        if ref["poly_trace_excess"] != 0.0:
            assert _close(rec["poly_trace_excess"], ref["poly_trace_excess"], 1e-12, 1e-6), (tag, who)
    # 2. GPU against oracle within what the field differences allow
    rho_g, u_g, C_g = g
    rho_o, u_o, C_o = r
    slack = 1.0 + 1e-6
    b = {}
    b["mass_A"] = np.abs(rho_g[0] - rho_o[0]).sum()
    b["mass_B"] = np.abs(rho_g[1] - rho_o[1]).sum() if rho_g.shape[0] == 2 else 0.0
    mg, mo = rho_g.sum(0) * u_g, rho_o.sum(0) * u_o
    for i, k in enumerate(("mom_x", "mom_y", "mom_z")):
        b[k] = np.abs(mg[i] - mo[i]).sum()
    dw = np.abs(ng["_w"] - no["_w"]).sum()
    b["W"] = dw
    b["max_u"] = np.sqrt(((u_g - u_o) ** 2).sum(0)).max()
    b["min_L2_minus_trC"] = np.abs(C_g[:3].sum(0) - C_o[:3].sum(0)).max()
    b["min_minor"] = np.abs(_minors(C_g) - _minors(C_o)).max()
    out = {}
    for k, bound in b.items():
        diff = abs(dg[k] - do[k])
        out[k] = (diff, bound)
        assert diff <= bound * slack + 1e-9 * max(abs(do[k]), 1e-300) + 1e-15, (tag, k, dg[k], do[k], bound)
    if no["W"] > 0:
        W = no["W"]
        arm = no["_rmax"] + 1.0
        for k in ("xc", "yc", "zc"):
            bound = 2.0 * dw * arm / W
            out[k] = (abs(dg[k] - do[k]), bound)
            assert out[k][0] <= bound, (tag, k, dg[k], do[k], bound)
        mb = 2.0 * dw * arm * arm / W
        for k in ("Mxx", "Myy", "Mzz", "Mxy", "Mxz", "Myz"):
            out[k] = (abs(dg[k] - do[k]), mb)
            assert out[k][0] <= mb, (tag, k, dg[k], do[k], mb)
        dM = math.sqrt((dg["Mxx"] - do["Mxx"]) ** 2 + (dg["Myy"] - do["Myy"]) ** 2 + 2 * (dg["Mxy"] - do["Mxy"]) ** 2)
        if no["_lam_gap"] > 10 * dM:
            dth = abs(dg["theta_deg"] - do["theta_deg"])
            dth = min(dth, abs(dth - 180.0))
            tb = math.degrees(2.0 * dM / no["_lam_gap"])
            out["theta_deg"] = (dth, tb)
            assert dth <= tb, (tag, "theta", dg["theta_deg"], do["theta_deg"], tb)
        # D = (sqrt l1 - sqrt l2)/(sqrt l1 + sqrt l2): |dD| <= |d l1| + |d l2| over the
        # smaller eigenvalue (first order), each eigenvalue moving by at most dM
        l2o = 0.5 * (no["Mxx"] + no["Myy"]) - 0.5 * no["_lam_gap"]
        if l2o > 10 * dM:
            db = 2.0 * dM / l2o
            out["D"] = (abs(dg["D"] - do["D"]), db)
            assert out["D"][0] <= db, (tag, "D", dg["D"], do["D"], db)
    assert dg["flags"] == do["flags"] == 0
    print(tag, "diag |gpu-oracle| (bound):",
          " ".join(f"{k}={v[0]:.1e}({v[1]:.1e})" for k, v in out.items()), flush=True)
