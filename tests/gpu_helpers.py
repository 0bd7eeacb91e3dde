"""Shared helpers of the GPU parity tests (comparison metrics and transfers)."""
import numpy as np

# Tolerances of the generator's outputs against the FP64 oracle, per particle
# and relative to the velocity's norm (components cross zero, so a component-
# wise relative error is meaningless): FP64 1e-13, FP32 4e-6.
TOL_FP64 = 1e-13
TOL_FP32 = 4e-6


def to_host(*tensors):
    return tuple(t.detach().cpu().numpy().astype(np.float64) for t in tensors)


def norm_rel_err(g, r):
    """max_i |v_gpu,i - v_ref,i|_2 / |v_ref,i|_2 for (vx, vy, vz) tuples of arrays."""
    gx, gy, gz = g
    rx, ry, rz = r
    d = np.sqrt((gx - rx) ** 2 + (gy - ry) ** 2 + (gz - rz) ** 2)
    nr = np.sqrt(rx ** 2 + ry ** 2 + rz ** 2)
    return float(np.max(d / nr)) if d.size else 0.0


def bits_equal(a, b):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(a, b))


def moments(vx, vy, vz):
    """Mean, variance and fourth central moment of each component and of v^2."""
    s2 = vx * vx + vy * vy + vz * vz
    out = {}
    for name, c in (("vx", vx), ("vy", vy), ("vz", vz), ("v2", s2)):
        m1 = c.mean()
        out[name] = {"mean": m1, "var": ((c - m1) ** 2).mean(), "m4": ((c - m1) ** 4).mean()}
    return out


def rel_errors(a, b):
    """Relative errors of var and m4; the error of a mean (near zero for the
    components) is expressed relative to the standard deviation."""
    out = {}
    for k in a:
        out[k] = {"mean_over_std": abs(a[k]["mean"] - b[k]["mean"]) / np.sqrt(b[k]["var"]),
                  "var": abs(a[k]["var"] / b[k]["var"] - 1), "m4": abs(a[k]["m4"] / b[k]["m4"] - 1)}
    return out
