"""Seeded synthetic volumes and filters shaped like the paper's workloads.

The paper evaluates ApplyFilter ("Gaussian blur to the structured volumes",
Sec. 4.3) on CT/medical and simulation data (Table 1: Heptane 302^3 UInt8,
DNS Float32, Richtmyer-Meshkov UInt8).  Those files are not available, so
these generators stand in for them.  Every random number comes from numpy's
PCG64 with a fixed seed, except the per-voxel noise of the two largest
volumes, which is drawn on the device from torch's seeded Philox generator.

This module holds no ApplyFilter arithmetic; both the GPU tests and the host
oracle consume what it returns.  Volumes are returned with shape (Z, Y, X)
(x fastest); filters with shape (k, k, k) indexed [c, b, a].
"""
import numpy as np

SEEDS = {"c1": 1001, "c2a": 2001, "c2b": 2002, "c2_blocks": 2003, "c3": 3001,
         "c3_blocks": 3002, "c3a_w": 3007, "c3b_w": 3009, "c4": 4001, "c5": 5001,
         "c5_blocks": 5002}


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- filters --

def gaussian_weights(k, sigma):
    """k^3 Gaussian sampled at integer offsets, normalised to sum 1 in FP64,
    then rounded to float32 (the float32 array is the filter)."""
    r = (k - 1) // 2
    o = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(o[:, None, None] ** 2 + o[None, :, None] ** 2
                 + o[None, None, :] ** 2) / (2.0 * sigma * sigma))
    return (g / g.sum()).astype(np.float32)


def box_int(k):
    """Integer box filter: all weights 1, divisor k^3."""
    return np.ones((k, k, k), np.int32), k ** 3


def random_l1(k, seed):
    """Dense N(0,1) weights normalised to unit L1 norm in FP64, then float32."""
    w = rng(seed).standard_normal((k, k, k))
    return (w / np.abs(w).sum()).astype(np.float32)


def sample_blocks(shape, n_random, seed, size=32):
    """Origins (x, y, z) of size^3 blocks of a (Z, Y, X) volume at which
    results are checked: the 8 corner blocks, then n_random blocks with
    origins uniform over the volume (seeded)."""
    Z, Y, X = shape
    bx, by, bz = min(size, X), min(size, Y), min(size, Z)
    out = [(x, y, z) for z in (0, Z - bz) for y in (0, Y - by) for x in (0, X - bx)]
    g = rng(seed)
    for _ in range(n_random):
        out.append((int(g.integers(0, X - bx + 1)), int(g.integers(0, Y - by + 1)),
                    int(g.integers(0, Z - bz + 1))))
    return out


# ---------------------------------------------------------------- volumes --

def uniform_f32(shape, seed):
    """i.i.d. U[0, 1) float32 voxels."""
    return rng(seed).random(shape, dtype=np.float32)


def _round_half_up_clamp(v, hi, dtype):
    return np.clip(np.floor(v + 0.5), 0, hi).astype(dtype)


def ct_phantom_u8(n=512, seed=SEEDS["c2a"], n_spheres=200):
    """CT-like uint8 phantom: N(40, 8^2) background plus solid spheres
    (centres U[0,n)^3, radius U[5,60], intensity U[100,255], later spheres
    painted over earlier ones), rounded half-up and clamped to 0..255."""
    g = rng(seed)
    vol = g.normal(40.0, 8.0, size=(n, n, n)).astype(np.float32)
    cen = g.uniform(0, n, size=(n_spheres, 3))
    rad = g.uniform(5, 60, size=n_spheres)
    val = g.uniform(100, 255, size=n_spheres)
    for (cx, cy, cz), rr, vv in zip(cen, rad, val):
        lo = [max(0, int(np.floor(c - rr))) for c in (cz, cy, cx)]
        hi = [min(n, int(np.ceil(c + rr)) + 1) for c in (cz, cy, cx)]
        zz, yy, xx = np.ogrid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        m = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= rr * rr
        vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]][m] = vv
    return _round_half_up_clamp(vol, 255, np.uint8)


def _torch():
    import torch
    return torch


def smoothed_noise_f32(n=512, sigma=4.0, seed=SEEDS["c2b"], device=None):
    """N(0,1) white noise low-passed by a Gaussian of std sigma (applied as
    its Fourier transfer function), rescaled to zero mean and unit sd."""
    noise = rng(seed).standard_normal((n, n, n), dtype=np.float32)
    if device is None:
        f = np.fft.rfftn(noise)
        fz = np.fft.fftfreq(n)[:, None, None]
        fy = np.fft.fftfreq(n)[None, :, None]
        fx = np.fft.rfftfreq(n)[None, None, :]
        f *= np.exp(-2.0 * (np.pi * sigma) ** 2 * (fx ** 2 + fy ** 2 + fz ** 2))
        v = np.fft.irfftn(f, s=noise.shape)
        v = (v - v.mean()) / v.std()
        return v.astype(np.float32)
    torch = _torch()
    t = torch.from_numpy(noise).to(device)
    f = torch.fft.rfftn(t)
    fr = torch.fft.fftfreq(n, device=device)
    fx = torch.fft.rfftfreq(n, device=device)
    h = torch.exp(-2.0 * (np.pi * sigma) ** 2 * fx[None, None, :] ** 2) \
        * torch.exp(-2.0 * (np.pi * sigma) ** 2 * fr[None, :, None] ** 2) \
        * torch.exp(-2.0 * (np.pi * sigma) ** 2 * fr[:, None, None] ** 2)
    v = torch.fft.irfftn(f * h, s=t.shape)
    v = (v - v.mean()) / v.std()
    return v.float().contiguous()


def blob_field_f32(n=1024, n_blobs=64, seed=SEEDS["c3"], device=None,
                   shape=None):
    """Simulation-like field: sum_j a_j exp(-|p - c_j|^2 / (2 s_j^2)) with
    c_j U[0,n)^3, s_j U[10,120], a_j N(0,1), plus U(-0.01R, 0.01R) noise where
    R = max - min of the blob sum.  shape (Z, Y, X) overrides n^3."""
    Z, Y, X = shape if shape is not None else (n, n, n)
    g = rng(seed)
    cen = g.uniform(0, 1, size=(n_blobs, 3)) * np.array([X, Y, Z])
    wid = g.uniform(10, 120, size=n_blobs)
    amp = g.standard_normal(n_blobs)
    if device is None:
        xp, mk = np, (lambda a: a)
        v = np.zeros((Z, Y, X), np.float32)
    else:
        torch = _torch()
        xp = torch
        mk = (lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device))
        v = torch.zeros((Z, Y, X), dtype=torch.float32, device=device)
    ax = [np.arange(m, dtype=np.float64) for m in (X, Y, Z)]
    for (cx, cy, cz), s, a in zip(cen, wid, amp):
        ex = mk(np.exp(-(ax[0] - cx) ** 2 / (2 * s * s)).astype(np.float32))
        ey = mk(np.exp(-(ax[1] - cy) ** 2 / (2 * s * s)).astype(np.float32))
        ez = mk((a * np.exp(-(ax[2] - cz) ** 2 / (2 * s * s))).astype(np.float32))
        for z0 in range(0, Z, 128):  # bounded temporaries
            z1 = min(Z, z0 + 128)
            v[z0:z1] += ez[z0:z1, None, None] * (ey[:, None] * ex[None, :])[None]
    R = float(v.max() - v.min())
    un = g.uniform(-0.01 * R, 0.01 * R, size=(Z, Y, X)).astype(np.float32) \
        if device is None else None
    if device is None:
        v += un
        return v
    # The 1% noise for device-side volumes comes from numpy in z-chunks so the
    # same seed gives the same noise on any machine.
    for z0 in range(0, Z, 64):
        z1 = min(Z, z0 + 64)
        chunk = g.uniform(-0.01 * R, 0.01 * R, size=(z1 - z0, Y, X))
        v[z0:z1] += mk(chunk.astype(np.float32))
    return v


def gamma_u16_volumes(count=256, seed=SEEDS["c4"], lo=32, hi=256,
                      ks=(3, 5, 7)):
    """Batched workload: `count` uint16 volumes, each axis U{lo..hi},
    values gamma(shape 2, scale 2000) rounded and clamped to 65535, and a
    filter size per volume drawn from ks.  Returns (volumes, ks)."""
    g = rng(seed)
    dims = g.integers(lo, hi + 1, size=(count, 3))
    kk = g.choice(np.array(ks), size=count)
    vols = []
    for (X, Y, Z) in dims:
        v = g.gamma(2.0, 2000.0, size=(int(Z), int(Y), int(X)))
        vols.append(_round_half_up_clamp(v, 65535, np.uint16))
    return vols, [int(k) for k in kk]


def ellipsoid_phantom_u16(shape=(1024, 2048, 2048), n_ell=5000,
                          seed=SEEDS["c5"], device=None):
    """Multi-material uint16 phantom: background 0, n_ell solid ellipsoids
    (centres uniform, semi-axes U[4,64], uniformly random orientation,
    intensity U[500,60000], painted in order), then per-voxel noise with
    sd = sqrt(intensity), rounded half-up and clamped to 0..65535.
    shape is (Z, Y, X)."""
    Z, Y, X = shape
    g = rng(seed)
    cen = g.uniform(0, 1, size=(n_ell, 3)) * np.array([X, Y, Z])
    semi = g.uniform(4, 64, size=(n_ell, 3))
    q = g.standard_normal((n_ell, 4))  # uniform random rotations
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    val = g.uniform(500, 60000, size=n_ell)
    torch = _torch() if device is not None else None
    if torch is None:
        v = np.zeros((Z, Y, X), np.float32)
    else:
        v = torch.zeros((Z, Y, X), dtype=torch.float32, device=device)
    for (cx, cy, cz), (sa, sb, sc), (w_, x_, y_, z_), iv in zip(cen, semi, q, val):
        Rm = np.array([
            [1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - z_ * w_), 2 * (x_ * z_ + y_ * w_)],
            [2 * (x_ * y_ + z_ * w_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - x_ * w_)],
            [2 * (x_ * z_ - y_ * w_), 2 * (y_ * z_ + x_ * w_), 1 - 2 * (x_ * x_ + y_ * y_)]])
        ext = max(sa, sb, sc)
        lo = [max(0, int(np.floor(c - ext))) for c in (cx, cy, cz)]
        hi = [min(m, int(np.ceil(c + ext)) + 1) for c, m in ((cx, X), (cy, Y), (cz, Z))]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        # M = R diag(1/s^2) R^T ; inside if d^T M d <= 1
        M = Rm @ np.diag([1 / sa ** 2, 1 / sb ** 2, 1 / sc ** 2]) @ Rm.T
        dx = np.arange(lo[0], hi[0]) - cx
        dy = np.arange(lo[1], hi[1]) - cy
        dz = np.arange(lo[2], hi[2]) - cz
        if torch is None:
            DZ, DY, DX = np.meshgrid(dz, dy, dx, indexing="ij")
            qf = (M[0, 0] * DX * DX + M[1, 1] * DY * DY + M[2, 2] * DZ * DZ
                  + 2 * M[0, 1] * DX * DY + 2 * M[0, 2] * DX * DZ
                  + 2 * M[1, 2] * DY * DZ)
            v[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]][qf <= 1.0] = iv
        else:
            tx = torch.from_numpy(dx).to(device)[None, None, :]
            ty = torch.from_numpy(dy).to(device)[None, :, None]
            tz = torch.from_numpy(dz).to(device)[:, None, None]
            qf = (M[0, 0] * tx * tx + M[1, 1] * ty * ty + M[2, 2] * tz * tz
                  + 2 * M[0, 1] * tx * ty + 2 * M[0, 2] * tx * tz
                  + 2 * M[1, 2] * ty * tz)
            sub = v[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            sub[qf <= 1.0] = float(iv)
    if torch is None:
        noise = g.standard_normal((Z, Y, X), dtype=np.float32)
        v = v + noise * np.sqrt(v)
        return _round_half_up_clamp(v, 65535, np.uint16)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty((Z, Y, X), dtype=torch.int32, device=device)
    for z0 in range(0, Z, 64):  # chunked to bound temporaries
        z1 = min(Z, z0 + 64)
        sl = v[z0:z1]
        nz = torch.randn(sl.shape, generator=gen, device=device, dtype=torch.float32)
        sl = sl + nz * torch.sqrt(sl)
        out[z0:z1] = torch.clamp(torch.floor(sl + 0.5), 0, 65535).to(torch.int32)
    del v
    # int32 in [0, 65535] -> the same 16 bits, viewed as uint16
    return out.to(torch.int16).view(torch.uint16)
