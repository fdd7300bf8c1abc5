"""Seeded synthetic inputs: geometries, initial density fields and per-node
wetting-parameter fields.

This module holds no lattice Boltzmann arithmetic.  It only draws shapes and
initial conditions, so that the GPU library and the CPU oracle can be fed
the same inputs.  The coexistence densities rho_g, rho_l that an initial
field uses are passed in by the caller.

Randomness is a counter-based SplitMix64 (Steele, Lea & Flood 2014; Vigna's
published constants): value i of stream s under seed k is
mix(key(k, s) + (i + 1) * 0x9E3779B97F4A7C15).
"""
import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed, stream):
    with np.errstate(over="ignore"):
        k = np.uint64(seed) * _GAMMA + np.uint64(stream) * np.uint64(0xD1B54A32D192ED03)
    return _mix(k)


def splitmix_u64(seed, stream, count, start=0):
    i = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(_key(seed, stream) + (i + np.uint64(1)) * _GAMMA)


def uniform(seed, stream, count, lo=0.0, hi=1.0, start=0):
    """count doubles uniform on [lo, hi) from stream `stream` of `seed`."""
    u = (splitmix_u64(seed, stream, count, start) >> np.uint64(11)).astype(np.float64)
    return lo + (hi - lo) * u * (1.0 / 9007199254740992.0)


def normal(seed, stream, count):
    """Box-Muller normals from two uniform streams."""
    u1 = uniform(seed, stream, count)
    u2 = uniform(seed, stream + 1, count)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


# --------------------------------------------------------------------------
# geometry (node index n = x + nx*(y + ny*z); arrays are shaped [nz][ny][nx])
# --------------------------------------------------------------------------

def _min_image(d, n):
    return (d + n / 2.0) % n - n / 2.0


def _grid(shape):
    if len(shape) == 2:
        ny, nx = shape
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        return [x.astype(np.float64), y.astype(np.float64)]
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return [x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)]


def dist_periodic(shape, center):
    """Minimum-image distance of every node to `center` (x, y[, z])."""
    g = _grid(shape)
    dims = list(reversed(shape))
    d2 = np.zeros(shape)
    for k, c in enumerate(center):
        d = _min_image(g[k] - c, dims[k])
        d2 += d * d
    return np.sqrt(d2)


def disk_mask(shape, center, radius):
    """Staircase solid: a node is solid iff |x - c|^2 <= R^2 (ties solid)."""
    g = _grid(shape)
    dims = list(reversed(shape))
    d2 = np.zeros(shape)
    for k, c in enumerate(center):
        d = _min_image(g[k] - c, dims[k])
        d2 += d * d
    return (d2 <= radius * radius).astype(np.uint8)


def channel_mask(nx, ny):
    """Two solid plates (rows y = 0 and y = ny - 1) on a periodic lattice."""
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[0, :] = 1
    m[-1, :] = 1
    return m


def poisson_disk_cylinders(n, count, rmin, rmax, seed, gap=2.0, max_tries=200000):
    """Dart throwing of `count` non-overlapping periodic cylinders on an n x n
    lattice: centres uniform, radii uniform on [rmin, rmax]; a draw is kept
    when its minimum-image centre distance to every kept cylinder is at least
    r_i + r_j + gap.  Returns an array [count, 3] of (cx, cy, r)."""
    kept = []
    i = 0
    while len(kept) < count and i < max_tries:
        cx, cy, r = uniform(seed, 10, 3, start=3 * i)
        cx, cy, r = cx * n, cy * n, rmin + (rmax - rmin) * r
        i += 1
        ok = True
        for (x, y, rr) in kept:
            dx, dy = _min_image(cx - x, n), _min_image(cy - y, n)
            if dx * dx + dy * dy < (r + rr + gap) ** 2:
                ok = False
                break
        if ok:
            kept.append((cx, cy, r))
    if len(kept) < count:
        raise RuntimeError(f"only {len(kept)} of {count} cylinders placed")
    return np.array(kept)


def cylinders_mask(n, cyl):
    """Solid mask and label field (index of the cylinder owning each solid
    node, -1 for fluid) of periodic cylinders on an n x n lattice."""
    mask = np.zeros((n, n), dtype=np.uint8)
    label = np.full((n, n), -1, dtype=np.int32)
    for k, (cx, cy, r) in enumerate(cyl):
        x0, x1 = int(math.floor(cx - r)) - 1, int(math.ceil(cx + r)) + 2
        y0, y1 = int(math.floor(cy - r)) - 1, int(math.ceil(cy + r)) + 2
        ys = np.arange(y0, y1)
        xs = np.arange(x0, x1)
        Y, X = np.meshgrid(ys, xs, indexing="ij")
        inside = (X - cx) ** 2 + (Y - cy) ** 2 <= r * r
        Yi, Xi = Y[inside] % n, X[inside] % n
        mask[Yi, Xi] = 1
        label[Yi, Xi] = k
    return mask, label


# --------------------------------------------------------------------------
# initial density fields
# --------------------------------------------------------------------------

def droplet_rho(shape, center, r0, rho_g, rho_l, width=3.0, solid=None):
    """tanh droplet: rho = (rl+rg)/2 - (rl-rg)/2 tanh(2 (r - r0) / W);
    solid nodes get 0."""
    r = dist_periodic(shape, center)
    rho = 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * (r - r0) / width)
    if solid is not None:
        rho = np.where(solid != 0, 0.0, rho)
    return rho


def add_noise(rho, amp, seed, solid=None, stream=7):
    """rho += U(-amp, amp) per node (node-indexed counter), fluid only."""
    u = uniform(seed, stream, rho.size, -amp, amp).reshape(rho.shape)
    out = rho + u
    if solid is not None:
        out = np.where(solid != 0, 0.0, out)
    return out


def _gauss_blur_periodic(field, sigma):
    shape = field.shape
    F = np.fft.rfftn(field)
    ks = [np.fft.fftfreq(s) for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    K = np.meshgrid(*ks, indexing="ij")
    k2 = sum(k * k for k in K)
    return np.fft.irfftn(F * np.exp(-2.0 * (np.pi ** 2) * (sigma ** 2) * k2), s=shape,
                         axes=tuple(range(len(shape))))


def blob_rho(shape, seed, rho_g, rho_l, solid=None, sigma=16.0, sigma2=1.5):
    """Random liquid/gas blobs: white noise -> periodic Gaussian blur (sigma)
    -> threshold at the fluid median (about half liquid) -> blur the
    indicator (sigma2) -> rho = rho_g + (rho_l - rho_g) H."""
    n = int(np.prod(shape))
    noise = normal(seed, 20, n).reshape(shape)
    sm = _gauss_blur_periodic(noise, sigma)
    fluid = np.ones(shape, bool) if solid is None else (solid == 0)
    thr = np.median(sm[fluid])
    H = _gauss_blur_periodic((sm > thr).astype(np.float64), sigma2)
    H = np.clip(H, 0.0, 1.0)
    rho = rho_g + (rho_l - rho_g) * H
    if solid is not None:
        rho = np.where(solid != 0, 0.0, rho)
    return rho


# --------------------------------------------------------------------------
# wetting-parameter fields: (phi, drho) on every solid node.  Each side
# gathers them at its own wall nodes.
# --------------------------------------------------------------------------

def angle_to_params(theta_deg, table):
    """Map prescribed angles to (phi, drho) by monotone linear interpolation
    in a calibration table {"theta": [...], "phi": [...], "drho": [...]}
    sorted by theta.  A table whose rows hold either phi >= 1 with drho = 0
    (below the standard-case angle) or phi = 1 with drho >= 0 (above it),
    with the standard case itself as a row, keeps that split."""
    th = np.asarray(table["theta"], dtype=np.float64)
    ph = np.asarray(table["phi"], dtype=np.float64)
    dr = np.asarray(table["drho"], dtype=np.float64)
    t = np.asarray(theta_deg, dtype=np.float64)
    return np.interp(t, th, ph), np.interp(t, th, dr)


def param_field(label, per_label_phi, per_label_drho):
    phi = np.ones(label.shape)
    drho = np.zeros(label.shape)
    m = label >= 0
    phi[m] = np.asarray(per_label_phi)[label[m]]
    drho[m] = np.asarray(per_label_drho)[label[m]]
    return phi, drho


def smooth_angle_profile(seed, n_modes=4):
    """Coefficients of g(beta) = sum_k a_k cos(k beta) + b_k sin(k beta),
    a_k, b_k ~ N(0, 1)/k, scaled so max |g| = 1 (sampled on a fine grid)."""
    z = normal(seed, 30, 2 * n_modes)
    k = np.arange(1, n_modes + 1)
    a, b = z[:n_modes] / k, z[n_modes:] / k
    beta = np.linspace(0.0, 2.0 * np.pi, 4096, endpoint=False)
    g = (a[:, None] * np.cos(k[:, None] * beta) + b[:, None] * np.sin(k[:, None] * beta)).sum(0)
    s = 1.0 / np.max(np.abs(g))
    return a * s, b * s


def eval_angle_profile(coef, beta):
    a, b = coef
    k = np.arange(1, len(a) + 1)
    beta = np.asarray(beta, dtype=np.float64)
    return (a[:, None] * np.cos(k[:, None] * beta[None]) +
            b[:, None] * np.sin(k[:, None] * beta[None])).sum(0)
