"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generation only - none of the multigrid or LPT
arithmetic.  Tests, the bench and the oracle checks all take their inputs from
here, so both the HIP path and the oracle see the same arrays.

Density fields follow Section 2.1 ("k-space sampling"): Gaussian white noise
mu ~ N(0,1) per cell, Fourier transformed, multiplied by sqrt(P(k)) and
transformed back.  The spectra are stand-ins for Boltzmann-code transfer
functions, which are not available here:

* BBKS (Bardeen, Bond, Kaiser & Szalay 1986) transfer function with shape
  parameter Gamma, P(k) = k T^2(k) (n_s = 1) - periodic single levels and
  zoom hierarchies;
* a pure power law P(k) = k^n with n in [-2.5, -1.5] - batched instances.

Nested fields (a stand-in for the paper's multi-scale convolution of
Section 2.3): level p is the conservative tri-cubic interpolation of level
p-1 (Section 2.3.4: tri-cubic, then each group of 8 children shifted so that
its mean equals the parent) plus fresh small-scale power s_p sampled on the
patch from its own seeded noise, keeping only modes above the parent's Nyquist
frequency, with s_p's own 8-child means removed (so the coarse-consistency
constraint "children average to the parent" of Section 2.3.1 holds exactly).
Amplitudes use one constant alpha for all levels, with sqrt(P/h^3) per-cell
normalisation so that refined noise carries 8x the variance of its parent,
as the Hoffman-Ribak refinement of Section 2.3.1 requires.
"""

import numpy as np

BOX = 100.0           # box length in Mpc/h
DELTA_RMS = 0.1       # rms of the base density field
GAMMA = 0.2           # BBKS shape parameter

SEED_C1 = 1103001
SEED_C2 = 1103002
SEED_C3 = 1103003
SEED_C4 = 1103004
SEED_C5 = 1103005


def bbks_transfer(k, gamma=GAMMA):
    q = np.asarray(k, dtype=np.float64) / gamma
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.log1p(2.34 * q) / (2.34 * q) * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3
                                              + (6.71 * q) ** 4) ** -0.25
    return np.where(q > 0, t, 1.0)


def spectrum_bbks(k):
    return k * bbks_transfer(k) ** 2


def spectrum_power_law(n):
    def P(k):
        with np.errstate(divide="ignore"):
            return np.where(k > 0, np.power(np.where(k > 0, k, 1.0), n), 0.0)
    return P


def _kgrid(shape, h):
    ks = [2.0 * np.pi * np.fft.fftfreq(n, d=h) for n in shape[:-1]]
    ks.append(2.0 * np.pi * np.fft.rfftfreq(shape[-1], d=h))
    return np.meshgrid(*ks, indexing="ij")


def _sample(mu, h, P, kmask=None):
    """irfftn(rfftn(mu) * sqrt(P(|k|)/h^3)), zero mode removed."""
    kx, ky, kz = _kgrid(mu.shape, h)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.sqrt(np.maximum(P(kk), 0.0) / h ** 3)
    amp[0, 0, 0] = 0.0
    if kmask is not None:
        amp = amp * kmask(kx, ky, kz)
    return np.fft.irfftn(np.fft.rfftn(mu) * amp, s=mu.shape, axes=(0, 1, 2))


def gaussian_field(N, seed, box=BOX, spectrum=spectrum_bbks, rms=DELTA_RMS, return_alpha=False):
    """Periodic N^3 density field with the given spectrum, rescaled to the given rms."""
    h = box / N
    mu = np.random.default_rng(seed).standard_normal((N, N, N))
    d = _sample(mu, h, spectrum)
    alpha = rms / np.sqrt(np.mean(d * d))
    d *= alpha
    return (d, alpha) if return_alpha else d


# ----------------------------------------------------------------------------- nested fields

_CUBIC_W = np.array([-7.0, 105.0, 35.0, -5.0]) / 128.0   # Lagrange cubic at +1/4 through -1, 0, 1, 2


def _cubic_axis(c, axis, lo_pad):
    """Tri-cubic step along one axis: coarse values (padded by lo_pad=2 each side) -> children."""
    c = np.moveaxis(c, axis, 0)
    m = c.shape[0] - 2 * lo_pad
    out = np.empty((2 * m,) + c.shape[1:])
    for I in range(m):
        j = I + lo_pad
        # child 2I at -1/4 mirrors the +1/4 weights through nodes +1, 0, -1, -2
        out[2 * I] = (_CUBIC_W[0] * c[j + 1] + _CUBIC_W[1] * c[j] + _CUBIC_W[2] * c[j - 1]
                      + _CUBIC_W[3] * c[j - 2])
        out[2 * I + 1] = (_CUBIC_W[0] * c[j - 1] + _CUBIC_W[1] * c[j] + _CUBIC_W[2] * c[j + 1]
                          + _CUBIC_W[3] * c[j + 2])
    return np.moveaxis(out, 0, axis)


def conservative_tricubic(parent, off, n, periodic):
    """Children of parent[off : off + n/2] by tri-cubic interpolation, 8-child means fixed."""
    idx = [np.arange(off[a] - 2, off[a] + n[a] // 2 + 2) for a in range(3)]
    if periodic:
        idx = [np.mod(i, parent.shape[a]) for a, i in enumerate(idx)]
    c = parent[np.ix_(*idx)]
    for a in range(3):
        c = _cubic_axis(c, a, 2)          # other axes stay padded until their turn
    fine = c
    nx, ny, nz = n
    pc = parent[np.ix_(*[np.mod(np.arange(off[a], off[a] + n[a] // 2), parent.shape[a]) for a in range(3)])]
    m8 = fine.reshape(nx // 2, 2, ny // 2, 2, nz // 2, 2).mean(axis=(1, 3, 5))
    corr = pc - m8
    return fine + np.repeat(np.repeat(np.repeat(corr, 2, 0), 2, 1), 2, 2)


def nested_fields(N0, patches, seed, box=BOX, spectrum=spectrum_bbks, rms=DELTA_RMS):
    """Density on a periodic N0^3 base plus nested patches [(n3, off3), ...].

    Returns a list of arrays (base first).  Each patch's 8-child means equal the
    parent cells they cover.
    """
    h0 = box / N0
    base, alpha = gaussian_field(N0, seed, box, spectrum, rms, return_alpha=True)
    out = [base]
    h_parent = h0
    for p, (n, off) in enumerate(patches, start=1):
        n = tuple(int(v) for v in n)
        h = h_parent / 2.0
        coarse = conservative_tricubic(out[-1], off, n, periodic=(p == 1))
        mu = np.random.default_rng(seed + p).standard_normal(n)
        kny = np.pi / h_parent

        def kmask(kx, ky, kz, kny=kny):
            return (np.maximum(np.maximum(np.abs(kx), np.abs(ky)), np.abs(kz)) > kny).astype(np.float64)

        s = alpha * _sample(mu, h, spectrum, kmask)
        s8 = s.reshape(n[0] // 2, 2, n[1] // 2, 2, n[2] // 2, 2).mean(axis=(1, 3, 5))
        s = s - np.repeat(np.repeat(np.repeat(s8, 2, 0), 2, 1), 2, 2)
        out.append(coarse + s)
        h_parent = h
    return out


# ----------------------------------------------------------------------------- multi-scale convolution inputs

def radial_transfer_table(alpha, h_finest, spectrum=spectrum_bbks, r_max=192.0, count=1 << 18):
    """The real-space transfer function T(r) = (1 / 2 pi^2) int T~(k) k^2 sin(kr) / (kr) dk of
    T~(k) = alpha sqrt(P(k)) exp(-(k / k_c)^2 / 2), tabulated at r = i dr (i < count,
    dr = r_max / count); returns (table, dr).

    This is input data, like P(k) itself: the paper obtains T(r) once from a Boltzmann code's
    transfer function with FFTlog.  Here a discrete sine transform on the uniform k grid
    k_j = j pi / r_max does the one-dimensional integral; the Gaussian cut at k_c = 2 pi / h_finest
    (the sub-cell Nyquist of the finest grid) keeps the integral finite.
    """
    dr = r_max / count
    dk = np.pi / r_max
    k = np.arange(count) * dk
    kc = 2.0 * np.pi / h_finest
    g = alpha * np.sqrt(np.maximum(spectrum(k), 0.0)) * np.exp(-0.5 * (k / kc) ** 2)
    g[0] = 0.0
    a = g * k
    ext = np.zeros(2 * count)
    ext[:count] = a
    ext[count + 1:] = -a[1:][::-1]
    s = -0.5 * np.imag(np.fft.fft(ext))[:count]          # sum_j a_j sin(pi i j / count)
    r = np.arange(count) * dr
    table = np.empty(count)
    table[1:] = s[1:] * dk / (2.0 * np.pi ** 2 * r[1:])
    table[0] = np.sum(g * k * k) * dk / (2.0 * np.pi ** 2)
    return table, dr


def multiscale_noise(N0, patches, seed):
    """Unit normals for the multi-scale convolution: N0^3 on the base, (2 n)^3 on every patch's
    padded domain (the patch centred in twice its size)."""
    rng = np.random.default_rng(seed)
    out = [rng.standard_normal((N0,) * 3)]
    for n, _ in patches:
        out.append(rng.standard_normal(tuple(2 * int(v) for v in n)))
    return out


def c3_multiscale_input(n_base=128, n_patch=128, depth=3, seed=SEED_C3):
    """The C3 geometry with the inputs of the multi-scale convolution: (patches, table, dr, xi).
    The amplitude is the one that gives the k-space sampled base field of this spectrum the rms
    DELTA_RMS."""
    patches = c3_layout(n_base, n_patch, depth)
    _, alpha = gaussian_field(n_base, seed, return_alpha=True)
    h_finest = BOX / n_base / 2 ** depth
    table, dr = radial_transfer_table(alpha, h_finest)
    return patches, table, dr, multiscale_noise(n_base, patches, seed + 17)


# ----------------------------------------------------------------------------- workloads

def c1_input():
    """64^3 periodic, BBKS, seed 1103001."""
    return gaussian_field(64, SEED_C1)


def c2_input():
    """256^3 periodic, BBKS, seed 1103002."""
    return gaussian_field(256, SEED_C2)


def c3_layout(n_base=128, n_patch=128, depth=3):
    """Base n_base^3 plus `depth` centred n_patch^3 patches at 2x finer spacing each."""
    patches = []
    parent = n_base
    for _ in range(depth):
        off = (parent - n_patch // 2) // 2
        patches.append(((n_patch,) * 3, (off,) * 3))
        parent = n_patch
    return patches


def c3_input(n_base=128, n_patch=128, depth=3):
    patches = c3_layout(n_base, n_patch, depth)
    return patches, nested_fields(n_base, patches, SEED_C3)


def c4_instances(count=64, seed=SEED_C4):
    """Batched periodic instances: (N, spectral index n, noise seed) per instance."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice([32, 48, 64, 96, 128], size=count)
    slopes = rng.uniform(-2.5, -1.5, size=count)
    return [(int(N), float(ns), seed * 1000 + i) for i, (N, ns) in enumerate(zip(sizes, slopes))]


def c4_field(N, slope, noise_seed):
    return gaussian_field(N, noise_seed, spectrum=spectrum_power_law(slope))


def c5_requests(count=600, rate=20.0, seed=SEED_C5):
    """Serving arrivals: Poisson(rate) times, base in {64,128,256}, depth 0-3 patches of 64-128."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    reqs = []
    for i in range(count):
        N0 = int(rng.choice([64, 128, 256]))
        depth = int(rng.integers(0, 4))
        patches = []
        parent = N0
        for _ in range(depth):
            choices = [m for m in (64, 96, 128) if m <= parent]
            n = int(rng.choice(choices))
            off = (parent - n // 2) // 2
            patches.append(((n,) * 3, (off,) * 3))
            parent = n
        order = 2 if rng.random() < 0.5 else 1
        reqs.append(dict(id=i, t=float(t[i]), N0=N0, patches=patches, order=order,
                         seed=seed * 1000 + i))
    return reqs
