"""Seeded synthetic workloads for the subspace-tracking step (NumPy only).

This module simulates the scanner and the ground truth: factor and phantom
image sequences, their k-space frames, Cartesian sampling masks and noise.  It
holds none of the reconstruction method's arithmetic, imports nothing from the
GPU library or from any reference implementation, and is the only code that
both the GPU path's tests and the FP64 reference checker consume (as inputs).

Every generator takes an explicit ``numpy.random.Generator``; ``rng_for`` gives
the seeded streams the configurations use:
``numpy.random.SeedSequence([1609, 4104, config, sequence, stream])``.

Workloads (the paper's data sets are in-vivo cardiac cine scans that are not
available, so these stand in for them):

* ``lowrank_sequence``   -- X_t = A* diag(gamma*_t) B*^T with A*, B* i.i.d. CN(0, 1),
  gamma*_{t,r} = sin(2 pi t / P_r + phi_r) + eps (P_r ~ U[5, 15], phi_r ~ U[0, 2 pi),
  eps ~ N(0, 0.01) in variance), sampled at uniformly random k-space points.
* ``phantom_sequence``   -- a cardiac-like cine: six additive ellipses (one body
  ellipse, two whose semi-axes breathe by 10 % with period 25 frames), 4 x 4
  supersampled, times a smooth degree-2 phase map.
* ``vd_line_mask``       -- variable-density Cartesian phase-encode lines: a fully
  sampled centre block plus lines drawn without replacement with weight
  |f|^alpha, alpha = -1, f the signed distance from the centre line (Sec. VI).
* ``kspace``             -- the orthonormal 2-D FFT of a frame (``numpy.fft``),
  i.e. what the scanner would measure, before noise.
"""

import numpy as np

__all__ = [
    "rng_for", "cn", "lowrank_truth", "lowrank_frame", "point_mask", "kspace",
    "signed_freq", "vd_line_mask", "PhantomSpec", "phantom_spec", "phantom_frame",
    "init_factors", "LineFrame", "PointFrame", "config1", "config2", "config3_kspace",
    "mixed_batch_specs", "phantom_bank", "serving_specs",
]


def rng_for(config, sequence=0, stream=0):
    """Independent seeded generator for (configuration, sequence, stream)."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([1609, 4104, int(config), int(sequence), int(stream)])))


def cn(rng, shape, var=1.0):
    """Circular complex Gaussian CN(0, var): real and imaginary parts N(0, var/2)."""
    s = np.sqrt(var / 2.0)
    return rng.normal(0.0, s, shape) + 1j * rng.normal(0.0, s, shape)


def kspace(X):
    """Orthonormal forward 2-D FFT (exp(-2 pi i k n / N), DC at index 0)."""
    return np.fft.fft2(np.asarray(X, dtype=np.complex128), norm="ortho")


def signed_freq(n):
    """Signed frequency f of each k-space row: i for i < n/2, else i - n."""
    i = np.arange(n)
    return np.where(i < (n + 1) // 2, i, i - n)


# ----------------------------------------------------------------------------- low rank
def lowrank_truth(n1, n2, r, T, rng):
    """A*, B* ~ CN(0, 1) and the temporal codes gamma*[t] for t = 1..T (row t-1)."""
    A = cn(rng, (n1, r))
    B = cn(rng, (n2, r))
    periods = rng.uniform(5.0, 15.0, r)
    phases = rng.uniform(0.0, 2.0 * np.pi, r)
    t = np.arange(1, T + 1, dtype=np.float64)[:, None]
    G = np.sin(2.0 * np.pi * t / periods[None, :] + phases[None, :])
    G = G + rng.normal(0.0, 0.1, (T, r))
    return A, B, G.astype(np.complex128)


def lowrank_frame(A, B, g):
    """The truth frame A* diag(g) B*^T (image domain)."""
    return (A * g[None, :]) @ B.T


def point_mask(n1, n2, count, rng):
    """Exactly ``count`` of the n1*n2 entries, uniformly without replacement."""
    m = np.zeros(n1 * n2, dtype=bool)
    m[rng.choice(n1 * n2, size=count, replace=False)] = True
    return m.reshape(n1, n2)


# ----------------------------------------------------------------------------- phantom
class PhantomSpec:
    """Ellipse parameters and phase map of one cine sequence."""

    def __init__(self, n1, n2, centres, axes, angles, intens, dyn_phase, phase_coef):
        self.n1, self.n2 = n1, n2
        self.centres, self.axes, self.angles = centres, axes, angles
        self.intens, self.dyn_phase, self.phase_coef = intens, dyn_phase, phase_coef


def phantom_spec(n1, n2, rng, n_ellipses=6):
    """Random cardiac-like phantom: ellipse 0 is the body, 1 and 2 breathe."""
    centres = rng.uniform(-0.5, 0.5, (n_ellipses, 2))
    centres[0] = rng.uniform(-0.1, 0.1, 2)
    axes = rng.uniform(0.1, 0.5, (n_ellipses, 2))
    axes[0] = rng.uniform(0.7, 0.9, 2)
    angles = rng.uniform(0.0, np.pi, n_ellipses)
    intens = rng.uniform(0.2, 1.0, n_ellipses)
    dyn_phase = rng.uniform(0.0, 2.0 * np.pi, 2)
    phase_coef = rng.uniform(-np.pi / 4, np.pi / 4, 6)
    return PhantomSpec(n1, n2, centres, axes, angles, intens, dyn_phase, phase_coef)


def _grid(n, ss):
    # sub-pixel centres on [-1, 1): pixel p covers [-1 + 2p/n, -1 + 2(p+1)/n)
    p = np.arange(n)[:, None]
    s = (np.arange(ss)[None, :] + 0.5) / ss
    return (-1.0 + 2.0 * (p + s) / n).reshape(-1)


def _ellipse_coverage(spec, k, scale, ss):
    """Fraction of each pixel inside ellipse k (ss x ss sub-pixel samples),
    evaluated only on the pixels of the ellipse's bounding box."""
    cx, cy = spec.centres[k]
    a, b = spec.axes[k] * scale
    c, s = np.cos(spec.angles[k]), np.sin(spec.angles[k])
    wx = np.sqrt((a * c) ** 2 + (b * s) ** 2)
    wy = np.sqrt((a * s) ** 2 + (b * c) ** 2)
    out = np.zeros((spec.n1, spec.n2))
    r0 = max(0, int(np.floor((cy - wy + 1.0) * spec.n1 / 2.0)) - 1)
    r1 = min(spec.n1, int(np.ceil((cy + wy + 1.0) * spec.n1 / 2.0)) + 1)
    c0 = max(0, int(np.floor((cx - wx + 1.0) * spec.n2 / 2.0)) - 1)
    c1 = min(spec.n2, int(np.ceil((cx + wx + 1.0) * spec.n2 / 2.0)) + 1)
    if r0 >= r1 or c0 >= c1:
        return out
    yy = _grid(spec.n1, ss)[r0 * ss:r1 * ss, None]
    xx = _grid(spec.n2, ss)[None, c0 * ss:c1 * ss]
    dx, dy = xx - cx, yy - cy
    u = (dx * c + dy * s) / a
    v = (-dx * s + dy * c) / b
    inside = (u * u + v * v) <= 1.0
    out[r0:r1, c0:c1] = inside.reshape(r1 - r0, ss, c1 - c0, ss).mean(axis=(1, 3))
    return out


def phantom_frame(spec, t, ss=4, period=25.0, amplitude=0.1, _static_cache={}):
    """Complex image of frame t (t = 1, 2, ...)."""
    key = id(spec)
    cached = _static_cache.get(key)
    if cached is None or cached[0] is not spec:
        static = np.zeros((spec.n1, spec.n2))
        for k in range(len(spec.intens)):
            if k not in (1, 2):
                static += spec.intens[k] * _ellipse_coverage(spec, k, 1.0, ss)
        y = (-1.0 + 2.0 * (np.arange(spec.n1) + 0.5) / spec.n1)[:, None]
        x = (-1.0 + 2.0 * (np.arange(spec.n2) + 0.5) / spec.n2)[None, :]
        c = spec.phase_coef
        phase = c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
        cached = (spec, static, np.exp(1j * phase))
        _static_cache.clear()
        _static_cache[key] = cached
    _, static, ph = cached
    mag = static.copy()
    for n, k in enumerate((1, 2)):
        scale = 1.0 + amplitude * np.sin(2.0 * np.pi * t / period + spec.dyn_phase[n])
        mag += spec.intens[k] * _ellipse_coverage(spec, k, scale, ss)
    return mag * ph


def vd_line_mask(n1, n_lines, rng, n_center=16, alpha=-1.0):
    """Ascending int32 rows: a centre block of min(n_center, n_lines // 2) rows with
    signed frequency in [-nc/2, nc/2), plus the other rows drawn without
    replacement with probability proportional to |f|^alpha."""
    n_lines = int(min(max(n_lines, 1), n1))
    nc = int(min(n_center, n_lines // 2))
    f = signed_freq(n1)
    centre = (f >= -(nc // 2)) & (f < nc - nc // 2)
    if nc == 0:
        centre = f == 0
    chosen = np.nonzero(centre)[0]
    rest = np.nonzero(~centre)[0]
    k = n_lines - chosen.size
    if k > 0:
        w = np.abs(f[rest]).astype(np.float64) ** alpha
        extra = rng.choice(rest, size=k, replace=False, p=w / w.sum())
        chosen = np.concatenate([chosen, extra])
    return np.sort(chosen).astype(np.int32)


def init_factors(n1, n2, r, rng):
    """Random start A0 ~ CN(0, 1/n1), B0 ~ CN(0, 1/n2), complex64."""
    A0 = cn(rng, (n1, r), 1.0 / n1).astype(np.complex64)
    B0 = cn(rng, (n2, r), 1.0 / n2).astype(np.complex64)
    return A0, B0


# ----------------------------------------------------------------------------- frames
class LineFrame:
    """One acquired frame: ascending rows (int32) and their samples [rows, n2] c64."""

    def __init__(self, rows, y, truth=None):
        self.rows, self.y, self.truth = rows, y, truth


class PointFrame:
    """One acquired frame: boolean mask [n1, n2] and a full [n1, n2] c64 sample
    array that is zero off the mask."""

    def __init__(self, mask, y, truth=None):
        self.mask, self.y, self.truth = mask, y, truth


def config1(T=20, n=64, r=8, count=1024, sigma=0.01, exact=False, perturb=0.0):
    """Low-rank truth, uniformly random points (25 % of 64 x 64), noise sigma.

    exact=True: every point sampled, no noise, and the start factors are the
    true ones, plus i.i.d. CN(0, perturb^2) noise when perturb > 0."""
    rng_truth, rng_mask, rng_noise, rng_init = (rng_for(1, 0, s) for s in range(4))
    A, B, G = lowrank_truth(n, n, r, T, rng_truth)
    frames = []
    for t in range(1, T + 1):
        X = lowrank_frame(A, B, G[t - 1])
        K = kspace(X)
        if exact:
            mask = np.ones((n, n), dtype=bool)
            y = K
        else:
            mask = point_mask(n, n, count, rng_mask)
            y = np.where(mask, K + cn(rng_noise, (n, n), sigma * sigma), 0.0)
        frames.append(PointFrame(mask, y.astype(np.complex64), truth=X))
    if exact:
        A0, B0 = A, B
        if perturb > 0:
            rng_p = rng_for(1, 0, 4)
            A0 = A + cn(rng_p, A.shape, perturb * perturb)
            B0 = B + cn(rng_p, B.shape, perturb * perturb)
        A0, B0 = A0.astype(np.complex64), B0.astype(np.complex64)
    else:
        A0, B0 = init_factors(n, n, r, rng_init)
    return dict(n1=n, n2=n, r=r, frames=frames, A0=A0, B0=B0, truth=(A, B, G))


def config2(T=200, n1=256, n2=256, r=32, accel=8, sigma=0.005, t_warm=5, seq=0, config=2):
    """Ellipse phantom cine with variable-density lines; the first ``t_warm``
    frames are fully sampled (warm start)."""
    rng_ph, rng_mask, rng_noise, rng_init = (rng_for(config, seq, s) for s in range(4))
    spec = phantom_spec(n1, n2, rng_ph)
    L = int(round(n1 / accel))
    frames = []
    for t in range(1, T + 1):
        img = phantom_frame(spec, t)
        K = kspace(img)
        rows = np.arange(n1, dtype=np.int32) if t <= t_warm else vd_line_mask(n1, L, rng_mask)
        y = K[rows, :] + cn(rng_noise, (rows.size, n2), sigma * sigma)
        frames.append(LineFrame(rows, y.astype(np.complex64), truth=img))
    A0, B0 = init_factors(n1, n2, r, rng_init)
    return dict(n1=n1, n2=n2, r=r, frames=frames, A0=A0, B0=B0, spec=spec)


def config3_kspace(T=200, n1=256, n2=256, r=32, sigma=0.005, seq=0):
    """Full noisy k-space frames (complex64 [T, n1, n2]) of the phantom cine, for
    acquisition at device-drawn rows, plus the images and start factors."""
    rng_ph, _, rng_noise, rng_init = (rng_for(3, seq, s) for s in range(4))
    spec = phantom_spec(n1, n2, rng_ph)
    K = np.empty((T, n1, n2), dtype=np.complex64)
    imgs = np.empty((T, n1, n2), dtype=np.complex64)
    for t in range(1, T + 1):
        img = phantom_frame(spec, t)
        imgs[t - 1] = img
        K[t - 1] = kspace(img) + cn(rng_noise, (n1, n2), sigma * sigma)
    A0, B0 = init_factors(n1, n2, r, rng_init)
    return dict(n1=n1, n2=n2, r=r, kspace=K, images=imgs, A0=A0, B0=B0, spec=spec)


def mixed_batch_specs(n_seq=64, seed_config=4):
    """Shapes, ranks and accelerations of the mixed batch: equal shares of
    128 x 128, 192 x 160 and 256 x 256 in seeded order, R ~ U{16, 32, 64},
    acceleration ~ U{4, ..., 12}."""
    rng = rng_for(seed_config, 0, 99)
    shapes = [(128, 128), (192, 160), (256, 256)]
    pick = np.array([i % 3 for i in range(n_seq)])
    rng.shuffle(pick)
    out = []
    for s in range(n_seq):
        n1, n2 = shapes[pick[s]]
        out.append(dict(n1=n1, n2=n2, r=int(rng.choice([16, 32, 64])),
                        accel=int(rng.integers(4, 13)), seq=s))
    return out


def phantom_bank(n, frames, seq=0, sigma=0.005, config=5, n2=None):
    """Full noisy k-space frames (complex64 [frames, n, n2], n2 = n by default)
    of one phantom cine."""
    n2 = n if n2 is None else n2
    rng_ph, rng_noise = rng_for(config, seq, 0), rng_for(config, seq, 2)
    spec = phantom_spec(n, n2, rng_ph)
    K = np.empty((frames, n, n2), dtype=np.complex64)
    for t in range(1, frames + 1):
        K[t - 1] = kspace(phantom_frame(spec, t)) + cn(rng_noise, (n, n2), sigma * sigma)
    return K


def serving_specs(n_scans=128, rate=16.0, sizes=(128, 160, 192, 256, 320, 384), ranks=(16, 32, 48, 64),
                  seed_config=5):
    """Scans of the serving workload: Poisson arrivals at `rate` scans/s (the
    first at 0), size N (N x N frames) and rank R drawn uniformly per scan, and
    each scan's start factors A0 ~ CN(0, 1/N), B0 ~ CN(0, 1/N)."""
    rng = rng_for(seed_config, 0, 98)
    gaps = rng.exponential(1.0 / rate, size=n_scans)
    arrivals = np.concatenate([[0.0], np.cumsum(gaps[1:])])
    out = []
    for s in range(n_scans):
        n = int(rng.choice(sizes))
        r = int(rng.choice(ranks))
        A0, B0 = init_factors(n, n, r, rng_for(seed_config, s, 3))
        out.append(dict(scan=s, n=n, r=r, arrival=float(arrivals[s]), A0=A0, B0=B0))
    return out


def coil_maps(n1, n2, C, rng, width=0.8):
    """Synthetic sensitivity maps H_c [C, n1, n2] (complex64): smooth Gaussian
    magnitudes centred on a ring just outside the field of view, each with a
    linear phase, normalised so that sum_c |H_c|^2 = 1 at every pixel (the
    sum-of-squares normalisation the paper estimates its maps with)."""
    y = (np.arange(n1) - n1 / 2) / (n1 / 2)
    x = (np.arange(n2) - n2 / 2) / (n2 / 2)
    Y, X = np.meshgrid(y, x, indexing="ij")
    off = rng.uniform(0, 2 * np.pi)
    H = np.empty((C, n1, n2), dtype=np.complex128)
    for c in range(C):
        th = off + 2 * np.pi * c / C
        cy, cx = 1.2 * np.sin(th), 1.2 * np.cos(th)
        mag = np.exp(-((Y - cy) ** 2 + (X - cx) ** 2) / (2 * width ** 2))
        a, b = rng.uniform(-np.pi / 2, np.pi / 2, 2)
        H[c] = mag * np.exp(1j * (a * X + b * Y + rng.uniform(0, 2 * np.pi)))
    H /= np.sqrt(np.sum(np.abs(H) ** 2, axis=0))[None]
    return H.astype(np.complex64)


class CoilFrame:
    """One multi-coil frame: ascending rows (int32) and their samples at every
    coil [C, rows, n2] c64."""

    def __init__(self, rows, y, truth=None):
        self.rows, self.y, self.truth = rows, y, truth


def config_coils(T=20, n1=128, n2=128, r=16, C=8, accel=4, sigma=0.005, t_warm=2, seq=0, config=6):
    """The phantom cine seen through C coils: y_c = [F(H_c .* X_t)] at
    variable-density rows, plus CN(0, sigma^2) noise per coil (Sec. IV-B's
    model); the first t_warm frames are fully sampled."""
    rng_ph, rng_mask, rng_noise, rng_init, rng_coil = (rng_for(config, seq, s) for s in range(5))
    spec = phantom_spec(n1, n2, rng_ph)
    H = coil_maps(n1, n2, C, rng_coil)
    L = int(round(n1 / accel))
    frames = []
    for t in range(1, T + 1):
        img = phantom_frame(spec, t)
        rows = np.arange(n1, dtype=np.int32) if t <= t_warm else vd_line_mask(n1, L, rng_mask)
        Y = np.stack([kspace(H[c].astype(np.complex128) * img)[rows, :] for c in range(C)])
        Y = Y + cn(rng_noise, Y.shape, sigma * sigma)
        frames.append(CoilFrame(rows, Y.astype(np.complex64), truth=img))
    A0, B0 = init_factors(n1, n2, r, rng_init)
    return dict(n1=n1, n2=n2, r=r, C=C, H=H, frames=frames, A0=A0, B0=B0)
