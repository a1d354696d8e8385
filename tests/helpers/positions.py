"""Hand-made bead coordinates for density and sweep tests."""
import numpy as np


def face_adjacent_fp32(edge32, ks, rng, per_face=6):
    """FP32 coordinates on and next to the faces k * edge32 (a few ulps either
    side) plus random ones, as FP64 values."""
    xs = []
    for k in ks:
        f = np.float32(np.float64(k) * np.float64(edge32))
        v = f
        for _ in range(per_face):
            v = np.nextafter(v, np.float32(-np.inf))
        for _ in range(2 * per_face + 1):
            xs.append(float(v))
            v = np.nextafter(v, np.float32(np.inf))
    xs += [float(np.float32(v)) for v in rng.uniform(ks[0] * edge32, ks[-1] * edge32, size=200)]
    return np.array(xs)
