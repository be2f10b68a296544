"""Parity checks of GPU results against the FP64 oracle (test helper).

Every comparison asserts two bounds on the same arrays:
  * relative l2:   ||got - ref|| / ||ref|| < tol, the tolerance stated for
    the path (1e-4 for FP32 paths, 2e-3 with the BF16 dictionary, 1e-5 for a
    single operator application);
  * element-wise:  max |got - ref| <= C * tol * max |ref| with C = 10, so that
    an error confined to a few pixels (a wrong border row or column, one
    wrong plane) fails even when it hardly moves the global norm.
The PSNR of the difference (peak = max |ref|) is printed beside them.
"""
import numpy as np

C_ELEMENT = 10.0


def stats(got, ref):
    """(rel_l2, max_abs, psnr) of got against ref."""
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    d = g - r
    rel = float(np.linalg.norm(d) / np.linalg.norm(r))
    mx = float(np.abs(d).max()) if d.size else 0.0
    peak = float(np.abs(r).max()) if r.size else 0.0
    mse = float(np.mean(d * d)) if d.size else 0.0
    psnr = float("inf") if mse == 0.0 else 10.0 * np.log10(peak * peak / mse)
    return rel, mx, psnr


def check(got, ref, tol, label=""):
    """Assert both bounds; returns the relative l2 error."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (label, g.shape, r.shape)
    assert np.all(np.isfinite(g)), f"{label}: non-finite values"
    rel, mx, psnr = stats(g, r)
    peak = float(np.abs(r).max())
    print(f"  parity {label}: rel_l2 {rel:.3e} (< {tol:g}), max_abs {mx:.3e} "
          f"(<= {C_ELEMENT * tol * peak:.3e}), psnr {psnr:.1f} dB", flush=True)
    assert rel < tol, f"{label}: rel_l2 {rel:.3e} >= {tol:g}"
    assert mx <= C_ELEMENT * tol * peak, (
        f"{label}: max_abs {mx:.3e} > {C_ELEMENT:g} * {tol:g} * {peak:.3e}")
    return rel
