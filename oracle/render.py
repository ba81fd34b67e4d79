"""Volume rendering of a lattice spline along rays (oracle; test infrastructure only).

The paper measures its reconstructions inside a volume renderer (Sec. 5.1,
Volume Rendering): rays march through the whole volume at evenly spaced
samples, under a transfer function that leaves the volume mostly
transparent.  The paper fixes no compositing rule; this oracle takes the
standard front-to-back emission-absorption order, written out step by step
in FP64:

  for every sample j = 0, 1, ... along the ray (sample 0 nearest the viewer):
    f, grad f     <- the convolution sum and its gradient at the sample
    rgba          <- transfer function at f: entry 0 at f0, entry T-1 at f1,
                     linear between neighbouring entries, clamped outside
    shade         <- ambient + diffuse |grad f . d| / |grad f|, with d the unit
                     ray direction, or ambient + diffuse when |grad f| <= grad_eps
    C             <- C + (1 - A) alpha shade rgb
    A             <- A + (1 - A) alpha
    stop once A >= alpha_stop

f and grad f come from ConvolutionSumOracle at the sample positions the
caller passes in (the float32 positions every implementation sees).
"""

import numpy as np


def transfer(tf, f0, f1, f):
    """RGBA of the transfer function tf (T x 4) at values f (any shape)."""
    tf = np.asarray(tf, dtype=np.float64)
    T = tf.shape[0]
    s = (np.asarray(f, dtype=np.float64) - f0) * ((T - 1) / (f1 - f0))
    s = np.clip(np.nan_to_num(s, nan=0.0), 0.0, T - 1)
    i = np.minimum(np.floor(s).astype(np.int64), T - 2)
    w = (s - i)[..., None]
    return tf[i] * (1.0 - w) + tf[i + 1] * w


def composite(f, grad, direction, tf, f0, f1, ambient, diffuse, grad_eps, alpha_stop):
    """Front-to-back compositing of samples (rays x steps): f (R x S),
    grad (R x S x 3), direction (3,).  Returns (R x 4): colour, opacity."""
    f = np.asarray(f, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    R, S = f.shape
    out = np.zeros((R, 4))
    for r in range(R):
        C = np.zeros(3)
        A = 0.0
        for j in range(S):
            if A >= alpha_stop:
                break
            rgba = transfer(tf, f0, f1, f[r, j])
            g = grad[r, j]
            gn = np.linalg.norm(g)
            shade = ambient + diffuse * (abs(g @ d) / gn if gn > grad_eps else 1.0)
            w = (1.0 - A) * rgba[3]
            C = C + w * shade * rgba[:3]
            A = A + w
        out[r, :3] = C
        out[r, 3] = A
    return out


def render_rays(oracle, coeffs, positions, direction, tf, f0, f1, ambient=0.3, diffuse=0.7, grad_eps=1e-6,
                alpha_stop=2.0):
    """positions: (R x S x 3) sample positions along R rays (sample 0 first).
    Evaluates f and grad f with the convolution-sum oracle, then composites."""
    P = np.asarray(positions, dtype=np.float64)
    R, S, _ = P.shape
    f, g = oracle.eval(coeffs, P.reshape(-1, 3), want_grad=True)
    return composite(f.reshape(R, S), g.reshape(R, S, 3), direction, tf, f0, f1, ambient, diffuse, grad_eps,
                     alpha_stop)
