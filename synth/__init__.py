"""Seeded synthetic inputs for the pMSz correction.

These stand in for the paper's datasets (Perlin noise for the weak- and
strong-scaling studies of Sec. V-C; the real datasets of Sec. V-B / V-D are not
available) and for its compressors (SZ3 / ZFP, replaced by a uniform
quantisation proxy with the same error-bound guarantee).  The module holds no
arithmetic of the correction itself: it only makes (f, fhat, xi) triples.

Determinism: every random draw comes from numpy's PCG64 on the host; the heavy
arithmetic (Perlin lattice sums) runs in torch float64 with one IEEE operation
per tensor op, so the same seed gives the same bits on the CPU and on a GPU.
The Gaussian random field is synthesised on the host (numpy + scipy FFT) and
then moved wherever it is needed.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft
import torch

# --------------------------------------------------------------------------
# Improved Perlin gradient noise (K. Perlin, "Improving Noise", SIGGRAPH 2002):
# quintic fade, 12 cube-edge gradients selected by a hashed lattice corner.
# The permutation is a seeded shuffle of 0..255 rather than the published one.
# --------------------------------------------------------------------------


def _fade(t):
    # 6t^5 - 15t^4 + 10t^3, one rounding per op
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _lerp(t, a, b):
    return a + t * (b - a)


def _grad(h, x, y, z):
    h = h & 15
    u = torch.where(h < 8, x, y)
    v = torch.where(h < 4, y, torch.where((h == 12) | (h == 14), x, z))
    u = torch.where((h & 1) == 0, u, -u)
    v = torch.where((h & 2) == 0, v, -v)
    return u + v


def _noise3(perm, x, y, z):
    fx, fy, fz = torch.floor(x), torch.floor(y), torch.floor(z)
    X = fx.to(torch.int64) & 255
    Y = fy.to(torch.int64) & 255
    Z = fz.to(torch.int64) & 255
    x, y, z = x - fx, y - fy, z - fz
    u, v, w = _fade(x), _fade(y), _fade(z)
    p = perm
    A = p[X] + Y
    AA = p[A] + Z
    AB = p[A + 1] + Z
    B = p[X + 1] + Y
    BA = p[B] + Z
    BB = p[B + 1] + Z
    x1, y1, z1 = x - 1.0, y - 1.0, z - 1.0
    return _lerp(w,
                 _lerp(v, _lerp(u, _grad(p[AA], x, y, z), _grad(p[BA], x1, y, z)),
                       _lerp(u, _grad(p[AB], x, y1, z), _grad(p[BB], x1, y1, z))),
                 _lerp(v, _lerp(u, _grad(p[AA + 1], x, y, z1), _grad(p[BA + 1], x1, y, z1)),
                       _lerp(u, _grad(p[AB + 1], x, y1, z1), _grad(p[BB + 1], x1, y1, z1))))


def perlin3d(shape, octaves, cells, seed, device="cpu", slab=16):
    """Fractal Perlin noise on a (nz, ny, nx) grid, float64, min-max normalised
    to [0, 1].  ``cells`` lattice cells span the domain at octave 0; each octave
    doubles the frequency and halves the amplitude, and is sampled at voxel
    centres plus a seeded non-integer offset so no sample sits on the lattice."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    perm = rng.permutation(256).astype(np.int64)
    perm = torch.from_numpy(np.concatenate([perm, perm])).to(device)
    offsets = rng.uniform(0.0, 256.0, size=(octaves, 3))
    out = torch.empty((nz, ny, nx), dtype=torch.float64, device=device)
    xs = torch.arange(nx, dtype=torch.float64, device=device) + 0.5
    ys = torch.arange(ny, dtype=torch.float64, device=device) + 0.5
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        zs = torch.arange(z0, z1, dtype=torch.float64, device=device) + 0.5
        acc = torch.zeros((z1 - z0, ny, nx), dtype=torch.float64, device=device)
        amp = 1.0
        for o in range(octaves):
            fx = cells * (2 ** o) / nx
            fy = cells * (2 ** o) / ny
            fz = cells * (2 ** o) / nz
            X = (xs * fx + offsets[o, 0]).view(1, 1, nx).expand(z1 - z0, ny, nx)
            Y = (ys * fy + offsets[o, 1]).view(1, ny, 1).expand(z1 - z0, ny, nx)
            Z = (zs * fz + offsets[o, 2]).view(z1 - z0, 1, 1).expand(z1 - z0, ny, nx)
            acc = acc + _noise3(perm, X, Y, Z) * amp
            amp *= 0.5
        out[z0:z1] = acc
    lo = float(out.min())
    hi = float(out.max())
    scale = 1.0 / (hi - lo)
    out.sub_(lo).mul_(scale)
    return out


# --------------------------------------------------------------------------
# Quantisation proxy for an error-bounded lossy compressor: the value is
# replaced by the centre of its bin of width 2*eps, plus uniform noise of
# +-eps/2, then clipped back inside the bound with a margin that absorbs the
# final rounding to the field's type.
# --------------------------------------------------------------------------


def quantise_proxy(f, eps, seed, chunk=1 << 24):
    """f: torch or numpy array (float32 / float64).  Returns fhat of the same
    type, kind and device with |fhat - f| <= eps (checked by the library)."""
    is_torch = isinstance(f, torch.Tensor)
    ft = f if is_torch else torch.from_numpy(np.ascontiguousarray(f))
    dtype = ft.dtype
    info = np.finfo(np.float32 if dtype == torch.float32 else np.float64)
    fmax = float(ft.abs().max()) if ft.numel() else 0.0
    margin = eps * 2.0 ** -10 + 2.0 * float(np.spacing(info.dtype.type(fmax + eps)))
    if margin >= eps:
        raise ValueError("error bound %g too small for the value range in %s" % (eps, dtype))
    rng = np.random.default_rng(seed + 1)
    out = torch.empty_like(ft)
    flat_in = ft.reshape(-1)
    flat_out = out.reshape(-1)
    inv = 1.0 / (2.0 * eps)
    half = eps - margin
    for s in range(0, flat_in.numel(), chunk):
        e = min(flat_in.numel(), s + chunk)
        x = flat_in[s:e].to(torch.float64)
        q = torch.round(x * inv)
        c = q * (2.0 * eps)
        u = torch.from_numpy(rng.uniform(-0.5 * eps, 0.5 * eps, size=e - s)).to(x.device)
        y = c + u
        y = torch.minimum(torch.maximum(y, x - half), x + half)
        flat_out[s:e] = y.to(dtype)
    return out if is_torch else out.numpy()


# --------------------------------------------------------------------------
# 2D Gaussian-peak fields (batched and serving workloads).
# --------------------------------------------------------------------------


# exp(-x) for x >= 0 from +, -, * and exact power-of-two scaling only, so
# that the same inputs give the same bits on any host (a vectorised libm exp
# may pick a different code path on another CPU): Cody-Waite reduction
# x = k ln2 + r with ln2 split into a head with trailing zero bits and a tail,
# then a degree-13 Taylor polynomial of exp(-r) for |r| <= ln2 / 2 (truncation
# below 1e-17 relative).
_LN2_HI = float.fromhex("0x1.62e42feep-1")
_LN2_LO = float.fromhex("0x1.a39ef35793c76p-33")
_INV_LN2 = float.fromhex("0x1.71547652b82fep+0")
_EXP_COEF = [1.0 / math.factorial(n) for n in range(13, -1, -1)]


def exp_neg(x):
    x = np.asarray(x, dtype=np.float64)
    k = np.floor(x * _INV_LN2 + 0.5)
    r = (x - k * _LN2_HI) - k * _LN2_LO
    y = -r
    p = np.full_like(y, _EXP_COEF[0])
    for c in _EXP_COEF[1:]:
        p = p * y + c
    return np.ldexp(p, -k.astype(np.int64))


def gaussian_peaks2d(ny, nx, seed, device="cpu"):
    """Sum of 50..500 Gaussian bumps (sigma 2..20 px, amplitude 0.5..1, each
    evaluated in a +-4 sigma window) plus 1% white noise; float32, made on the
    host in binary64 and then moved to `device`.  Every draw comes from PCG64
    and the arithmetic uses only correctly rounded operations (exp_neg), so a
    seed gives the same bits on any host.  A bump is the outer product of its
    two one-dimensional profiles."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(50, 501))
    cx = rng.uniform(0, nx, k)
    cy = rng.uniform(0, ny, k)
    sig = rng.uniform(2.0, 20.0, k)
    amp = rng.uniform(0.5, 1.0, k)
    win = []
    for j in range(k):
        r = 4.0 * sig[j]
        x0, x1 = max(0, int(math.floor(cx[j] - r))), min(nx, int(math.ceil(cx[j] + r)) + 1)
        y0, y1 = max(0, int(math.floor(cy[j] - r))), min(ny, int(math.ceil(cy[j] + r)) + 1)
        win.append((x0, x1, y0, y1))
    # all one-dimensional profiles of the field in one evaluation
    xs = np.concatenate([np.arange(w[0], w[1], dtype=np.float64) - cx[j]
                         for j, w in enumerate(win)] + [np.zeros(0)])
    ys = np.concatenate([np.arange(w[2], w[3], dtype=np.float64) - cy[j]
                         for j, w in enumerate(win)] + [np.zeros(0)])
    sx = np.concatenate([np.full(max(w[1] - w[0], 0), 2.0 * sig[j] ** 2)
                         for j, w in enumerate(win)] + [np.zeros(0)])
    sy = np.concatenate([np.full(max(w[3] - w[2], 0), 2.0 * sig[j] ** 2)
                         for j, w in enumerate(win)] + [np.zeros(0)])
    ex = exp_neg(xs * xs / sx)
    ey = exp_neg(ys * ys / sy)
    h = np.zeros((ny, nx), dtype=np.float64)
    ox = oy = 0
    for j, (x0, x1, y0, y1) in enumerate(win):
        wx, wy = max(x1 - x0, 0), max(y1 - y0, 0)
        if wx and wy:
            h[y0:y1, x0:x1] += amp[j] * np.multiply.outer(ey[oy:oy + wy], ex[ox:ox + wx])
        ox += wx
        oy += wy
    rng_h = float(h.max() - h.min())
    noise = np.random.default_rng(int(rng.integers(1 << 62))).standard_normal((ny, nx))
    h += noise * (0.01 * max(rng_h, 1e-12))
    return torch.from_numpy(h.astype(np.float32)).to(device)


def batch_recipe(n_fields, seed, lo=256, hi=4096):
    """Sizes and bounds of the uneven 2D batch: nx and ny drawn independently
    log-uniform on [lo, hi]; relative bound from {1e-2, 1e-3, 1e-4}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_fields):
        nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        rel = float(rng.choice([1e-2, 1e-3, 1e-4]))
        out.append({"nx": nx, "ny": ny, "rel_eps": rel, "seed": int(rng.integers(1 << 31))})
    return out


def make_2d_case(nx, ny, rel_eps, seed, device="cpu"):
    """(f, fhat, xi) for one Gaussian-peak field, xi relative to the range of f."""
    f = gaussian_peaks2d(ny, nx, seed, device=device)
    rng_f = float(f.max()) - float(f.min())
    xi = rel_eps * rng_f
    fhat = quantise_proxy(f, xi, seed)
    return f, fhat, xi


def batch_cases(n_fields, seed, device="cpu", workers=None):
    """The uneven 2D batch of batch_recipe(n_fields, seed) as (f, fhat, xi)
    triples on `device`; the fields are made on the host by a thread pool
    (each field from its own seed, so the result does not depend on the
    number of threads)."""
    rec = batch_recipe(n_fields, seed)
    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        fs = list(ex.map(lambda c: gaussian_peaks2d(c["ny"], c["nx"], c["seed"]), rec))
    out = []
    for c, f in zip(rec, fs):
        f = f.to(device)
        xi = c["rel_eps"] * (float(f.max()) - float(f.min()))
        out.append((f, quantise_proxy(f, xi, c["seed"]), xi))
    return out


# --------------------------------------------------------------------------
# Gaussian random field with power spectrum k^-3 (FFT synthesis), float64.
# --------------------------------------------------------------------------


def _normal_slabs(shape, seed, slab=16, workers=None):
    """N(0, 1) values of the given (nz, ny, nx) shape, drawn slab by slab of
    `slab` z-planes, each slab from its own PCG64 stream spawned from `seed`,
    so that the values do not depend on how many threads draw them."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=np.float64)
    seqs = np.random.SeedSequence(seed).spawn((nz + slab - 1) // slab)

    def fill(k):
        z0, z1 = k * slab, min(nz, (k + 1) * slab)
        np.random.Generator(np.random.PCG64(seqs[k])).standard_normal(
            size=(z1 - z0, ny, nx), out=out[z0:z1])

    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fill, range(len(seqs))))
    return out


def grf3d(shape, seed, workers=None):
    """Gaussian random field with power spectrum |k|^-3 on the host, binary64,
    normalised to [0, 1] (torch CPU tensor).  White noise -> rfftn -> scale by
    |k|^-3/2 (integer wavenumbers, k = 0 removed) -> irfftn.  scipy's FFT
    computes each 1-D transform the same way whatever the worker count, so a
    seed gives the same bits on any x86-64 host with this software."""
    nz, ny, nx = shape
    workers = workers or min(16, os.cpu_count() or 1)
    W = sfft.rfftn(_normal_slabs(shape, seed, workers=workers), workers=workers,
                   overwrite_x=True)
    kz = sfft.fftfreq(nz, d=1.0 / nz)
    ky = sfft.fftfreq(ny, d=1.0 / ny)
    kx = sfft.rfftfreq(nx, d=1.0 / nx)
    for z0 in range(0, nz, 64):
        z1 = min(nz, z0 + 64)
        k2 = kz[z0:z1, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
        amp = np.zeros_like(k2)
        np.power(k2, -0.75, out=amp, where=k2 > 0)
        W[z0:z1] *= amp
    out = sfft.irfftn(W, s=(nz, ny, nx), workers=workers, overwrite_x=True)
    del W
    lo, hi = float(out.min()), float(out.max())
    out -= lo
    out *= 1.0 / (hi - lo)
    return torch.from_numpy(out)


# --------------------------------------------------------------------------
# Named workloads.
# --------------------------------------------------------------------------


def perlin_case(n, octaves, cells, eps, seed, dtype=torch.float32, device="cpu"):
    """(f, fhat, xi) for an n^3 Perlin field normalised to [0, 1] (range 1, so
    the relative and absolute bounds coincide)."""
    f = perlin3d((n, n, n), octaves, cells, seed, device=device).to(dtype)
    fhat = quantise_proxy(f, eps, seed)
    return f, fhat, eps


def small_perlin_case(device="cpu"):
    """64^3 float32, 4 octaves, 4 cells, eps = 1e-3, seed 1234."""
    return perlin_case(64, 4, 4, 1e-3, 1234, device=device)


def large_perlin_case(device="cpu"):
    """512^3 float32, 6 octaves, 8 cells, eps = 1e-4 (range 1), seed 512."""
    return perlin_case(512, 6, 8, 1e-4, 512, device=device)


def grf_case(shape=(768, 1024, 1024), rel_eps=1e-5, seed=1024, device="cpu"):
    """(f, fhat, xi) for a binary64 Gaussian random field with power spectrum
    k^-3, normalised to [0, 1]; xi = rel_eps * (max f - min f).  The default
    is the 1024 x 1024 x 768 large-field workload."""
    f = grf3d(shape, seed).to(device)
    xi = rel_eps * (float(f.max()) - float(f.min()))
    fhat = quantise_proxy(f, xi, seed)
    return f, fhat, xi
