"""Seeded synthetic inputs for the MPDATA step (numpy, FP64 generation).

This module holds no arithmetic of the advection scheme: it only draws the
five input fields (psi, u1, u2, u3, h) of the workloads the library is
measured and tested on.  Both the HIP path and the CPU oracle are fed from
here; neither is imported by this module.

Layout (shared by every generator): cell arrays are ``[nz][ny][nx]`` with x
fastest; face Courant arrays carry n+1 faces on their own axis,
``u1[nz][ny][nx+1]``, ``u2[nz][ny+1][nx]``, ``u3[nz+1][ny][nx]``, face ``i'``
lying between cells ``i'-1`` and ``i'``.  With periodic boundaries the last
face along an axis repeats the first one bit for bit.

The paper measures on a 240x240x128 and a 480x480x128 MPDATA domain in FP64
for 40 steps (section 6) and publishes no input data; these generators stand
in for that data with seeded fields of the shapes below:

* ``parity_small``  -- 32x32x16, FP64, periodic, 10 steps, constant Courant
  (0.3, 0.2, 0.1), h = 1, psi = 1 + Gaussian blob (sigma 4 cells) at the grid
  middle with a seeded jitter of the centre.
* ``rotation``      -- 512x256x64, periodic, solid-body rotation in x-y with
  max |u2| = 0.5, u3 = 0.1, h = 1 + three seeded sinusoids in [0.8, 1.2],
  psi = cone + slotted cube on a zero background.
* ``streamfunction``-- 1024x512x64, open boundaries, divergence-free x-y
  velocity from a seeded streamfunction quantised to 2**-16 (so u is exactly
  divergence-free in FP32 and FP64), max |u| = 0.4, h = 1, log-normal psi.
* ``batched_grids`` -- 96 uneven grids (nx, ny log-uniform in [32, 384], nz in
  [16, 64]), constant Courant per grid drawn in [-0.5, 0.5]^3 and kept only
  when |C1|+|C2|+|C3| <= 1, h = 1, psi = 1 + Gaussian blob.
* ``served_requests`` -- Poisson arrivals of rotation-flow requests with
  uneven dims, step counts and precisions.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BC_PERIODIC = 0
BC_OPEN = 1


@dataclasses.dataclass
class Fields:
    psi: np.ndarray
    u1: np.ndarray
    u2: np.ndarray
    u3: np.ndarray
    h: np.ndarray
    bc: int = BC_PERIODIC

    @property
    def shape(self):
        return self.psi.shape

    @property
    def cells(self) -> int:
        return int(self.psi.size)

    def astype(self, dtype) -> "Fields":
        """Round every field to ``dtype`` (the FP32 runs and their FP64
        oracle both start from these rounded values)."""
        return Fields(*(np.ascontiguousarray(a.astype(dtype)) for a in
                        (self.psi, self.u1, self.u2, self.u3, self.h)), bc=self.bc)

    def as_f64(self) -> "Fields":
        return self.astype(np.float64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def constant_courant(shape, c, dtype=np.float64):
    """Face arrays holding one Courant vector everywhere."""
    nz, ny, nx = shape
    u1 = np.full((nz, ny, nx + 1), c[0], dtype)
    u2 = np.full((nz, ny + 1, nx), c[1], dtype)
    u3 = np.full((nz + 1, ny, nx), c[2], dtype)
    return u1, u2, u3


def _centres(n):
    return np.arange(n, dtype=np.float64) + 0.5


def _min_image(d, n):
    return d - n * np.round(d / n)


def gaussian_blob(shape, centre, sigma, periodic=True):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    dx, dy, dz = x - centre[0], y - centre[1], z - centre[2]
    if periodic:
        dx, dy, dz = _min_image(dx, nx), _min_image(dy, ny), _min_image(dz, nz)
    return np.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * sigma * sigma))


# --------------------------------------------------------------- workloads

def parity_small(seed: int = 1001, shape=(16, 32, 32)) -> Fields:
    """Plain FP64 case: 32x32x16 periodic, constant Courant (0.3, 0.2, 0.1)."""
    rng = _rng(seed)
    nz, ny, nx = shape
    jitter = rng.uniform(-0.5, 0.5, 3)
    centre = (nx / 2 + jitter[0], ny / 2 + jitter[1], nz / 2 + jitter[2])
    psi = 1.0 + gaussian_blob(shape, centre, 4.0)
    u1, u2, u3 = constant_courant(shape, (0.3, 0.2, 0.1))
    return Fields(psi, u1, u2, u3, np.ones(shape), BC_PERIODIC)


def rotation(seed: int = 1002, shape=(64, 256, 512), u3_value=0.1) -> Fields:
    """Solid-body rotation about the x-y centre, max |u2| = 0.5."""
    rng = _rng(seed)
    nz, ny, nx = shape
    omega = 0.5 / (nx / 2 - 0.5)
    yc = _centres(ny) - ny / 2          # x-faces sit at cell-centre y
    xc = _centres(nx) - nx / 2          # y-faces sit at cell-centre x
    u1 = np.broadcast_to((-omega * yc)[None, :, None], (nz, ny, nx + 1)).copy()
    u2 = np.broadcast_to((omega * xc)[None, None, :], (nz, ny + 1, nx)).copy()
    u3 = np.full((nz + 1, ny, nx), u3_value)
    # density: 1 + (0.2/3) * sum of three seeded periodic sinusoids
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    h = np.ones(shape)
    choices = [(a, b, c) for a in range(3) for b in range(3) for c in range(3)
               if (a, b, c) != (0, 0, 0)]
    for _ in range(3):
        a, b, c = choices[rng.integers(len(choices))]
        phi = rng.uniform(0.0, 2.0 * math.pi)
        h += (0.2 / 3.0) * np.sin(2 * math.pi * (a * x / nx + b * y / ny + c * z / nz) + phi)
    # psi: cone and slotted cube on a zero background (positions scale with the grid)
    psi = np.zeros(shape)
    s = nx / 512.0
    cone_c = (128 * s, ny / 2, nz / 2)
    r = np.sqrt((x - cone_c[0]) ** 2 + (y - cone_c[1]) ** 2 + (z - cone_c[2]) ** 2)
    psi = np.maximum(psi, np.maximum(0.0, 1.0 - r / (24 * s)))
    cube_c = (384 * s, ny / 2, nz / 2)
    half = 24 * s
    inside = ((np.abs(x - cube_c[0]) <= half) & (np.abs(y - cube_c[1]) <= half)
              & (np.abs(z - cube_c[2]) <= min(half, nz / 2 - 1)))
    slot = (np.abs(x - cube_c[0]) < 4 * s) & (y > cube_c[1] - 8 * s)
    psi[inside & ~slot] = 1.0
    return Fields(psi, u1, u2, u3, h, BC_PERIODIC)


def divergent_rotation(seed: int = 1004, shape=(64, 256, 512), umax=0.35, amp=0.05) -> Fields:
    """The rotation workload made divergent: the solid-body flow scaled to
    max |u2| = umax plus a compressible part amp cos(2 pi f/n) on the faces of
    every axis (amp/2 along z), so every cell has a nonzero divergence; the
    outflow of a cell stays below the smallest h (0.8)."""
    f = rotation(seed, shape)
    nz, ny, nx = shape
    k = umax / 0.5
    u1 = f.u1 * k + amp * np.cos(2 * math.pi * np.arange(nx + 1) / nx)[None, None, :]
    u2 = f.u2 * k + amp * np.cos(2 * math.pi * np.arange(ny + 1) / ny)[None, :, None]
    u3 = f.u3 + 0.5 * amp * np.cos(2 * math.pi * np.arange(nz + 1) / nz)[:, None, None]
    # periodic: face n is face 0, bit for bit
    u1[..., nx] = u1[..., 0]
    u2[:, ny, :] = u2[:, 0, :]
    u3[nz] = u3[0]
    return Fields(f.psi, u1, u2, u3, f.h, BC_PERIODIC)


def streamfunction(seed: int = 1003, shape=(64, 512, 1024), umax=0.4) -> Fields:
    """Open domain, divergence-free x-y flow from a quantised streamfunction."""
    rng = _rng(seed)
    nz, ny, nx = shape
    xc = np.arange(nx + 1, dtype=np.float64)   # corner coordinates
    yc = np.arange(ny + 1, dtype=np.float64)
    zc = _centres(nz)
    Y, X = np.meshgrid(yc, xc, indexing="ij")      # (ny+1, nx+1)
    modes = []
    for _ in range(8):
        modes.append((rng.normal(), int(rng.integers(1, 5)), int(rng.integers(1, 5)),
                      int(rng.integers(0, 3)), rng.uniform(0, 2 * math.pi),
                      rng.uniform(0, 2 * math.pi)))
    psi_s = np.zeros((nz, ny + 1, nx + 1))
    for a, p, q, r, phi, theta in modes:
        plane = a * np.sin(2 * math.pi * (p * X / nx + q * Y / ny) + phi)
        prof = 1.0 + 0.5 * np.cos(2 * math.pi * r * zc / nz + theta)
        psi_s += plane[None, :, :] * prof[:, None, None]

    def velocities(s):
        u1 = s[:, 1:, :] - s[:, :-1, :]            # (nz, ny, nx+1)
        u2 = -(s[:, :, 1:] - s[:, :, :-1])         # (nz, ny+1, nx)
        return u1, u2

    u1, u2 = velocities(psi_s)
    scale = umax / max(np.abs(u1).max(), np.abs(u2).max())
    q = 2.0 ** -16
    psi_s = np.round(psi_s * scale / q) * q
    u1, u2 = velocities(psi_s)
    u3 = np.zeros((nz + 1, ny, nx))
    psi = np.exp(0.5 * rng.normal(size=shape))
    return Fields(np.ascontiguousarray(psi), np.ascontiguousarray(u1),
                  np.ascontiguousarray(u2), u3, np.ones(shape), BC_OPEN)


def batched_grid(g: int) -> Fields:
    """Grid ``g`` of the 96-grid batched workload (seed 4000 + g)."""
    rng = _rng(4000 + g)
    nx = int(np.rint(np.exp(rng.uniform(math.log(32), math.log(384)))))
    ny = int(np.rint(np.exp(rng.uniform(math.log(32), math.log(384)))))
    nz = int(np.rint(np.exp(rng.uniform(math.log(16), math.log(64)))))
    while True:
        c = rng.uniform(-0.5, 0.5, 3)
        if np.abs(c).sum() <= 1.0:
            break
    shape = (nz, ny, nx)
    sigma = max(2.0, min(shape) / 8.0)
    centre = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
    psi = 1.0 + gaussian_blob(shape, centre, sigma)
    u1, u2, u3 = constant_courant(shape, c)
    return Fields(psi, u1, u2, u3, np.ones(shape), BC_PERIODIC)


def batched_grids(n: int = 96):
    return [batched_grid(g) for g in range(n)]


def rotation_request(rng: np.random.Generator, nx: int, ny: int, nz: int,
                     sense: int) -> Fields:
    """Solid-body rotation about the grid centre, max component Courant 0.5,
    u3 = 0, h = 1, periodic, psi = 1 + Gaussian blob."""
    shape = (nz, ny, nx)
    omega = 0.5 / (max(nx, ny) / 2 - 0.5)
    yc = _centres(ny) - ny / 2
    xc = _centres(nx) - nx / 2
    u1 = np.broadcast_to((-sense * omega * yc)[None, :, None], (nz, ny, nx + 1)).copy()
    u2 = np.broadcast_to((sense * omega * xc)[None, None, :], (nz, ny + 1, nx)).copy()
    u3 = np.zeros((nz + 1, ny, nx))
    centre = (nx * rng.uniform(0.3, 0.7), ny * rng.uniform(0.3, 0.7), nz / 2)
    sigma = max(2.0, min(shape) / 8.0)
    psi = 1.0 + gaussian_blob(shape, centre, sigma)
    return Fields(psi, u1, u2, u3, np.ones(shape), BC_PERIODIC)


def rotation_request_device(req: "Request", device="cuda"):
    """The fields of ``req`` built directly in device memory with torch (same
    recipe as :func:`rotation_request`; values may differ from the numpy
    build in the last bits of exp).  Returns (psi, u1, u2, u3, h)."""
    import torch
    rng = _rng(req.field_seed)
    nz, ny, nx = req.shape
    centre = (nx * rng.uniform(0.3, 0.7), ny * rng.uniform(0.3, 0.7), nz / 2)
    sigma = max(2.0, min(req.shape) / 8.0)
    omega = 0.5 / (max(nx, ny) / 2 - 0.5)
    f64 = dict(dtype=torch.float64, device=device)
    yc = torch.arange(ny, **f64) + 0.5 - ny / 2
    xc = torch.arange(nx, **f64) + 0.5 - nx / 2
    u1 = (-req.sense * omega * yc)[None, :, None].expand(nz, ny, nx + 1)
    u2 = (req.sense * omega * xc)[None, None, :].expand(nz, ny + 1, nx)
    u3 = torch.zeros((nz + 1, ny, nx), **f64)
    h = torch.ones((nz, ny, nx), **f64)

    def d(n, c):
        v = torch.arange(n, **f64) + 0.5 - c
        return v - n * torch.round(v / n)

    dz, dy, dx = d(nz, centre[2]), d(ny, centre[1]), d(nx, centre[0])
    r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    psi = 1.0 + torch.exp(-r2 / (2.0 * sigma * sigma))
    dt = torch.float32 if req.fp32 else torch.float64
    return tuple(t.to(dt).contiguous() for t in (psi, u1, u2, u3, h))


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float       # seconds from the start of the run
    shape: tuple         # (nz, ny, nx)
    steps: int
    fp32: bool
    sense: int
    field_seed: int

    @property
    def cells(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    def fields(self) -> Fields:
        rng = _rng(self.field_seed)
        nz, ny, nx = self.shape
        f = rotation_request(rng, nx, ny, nz, self.sense)
        return f.astype(np.float32) if self.fp32 else f


def served_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 5000):
    """Poisson arrivals; dims log-uniform [32,256]^2 x [16,64], steps uniform
    in [10, 200], 70 % FP32 / 30 % FP64."""
    rng = _rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        nx = int(np.rint(np.exp(rng.uniform(math.log(32), math.log(256)))))
        ny = int(np.rint(np.exp(rng.uniform(math.log(32), math.log(256)))))
        nz = int(np.rint(np.exp(rng.uniform(math.log(16), math.log(64)))))
        steps = int(rng.integers(10, 201))
        fp32 = bool(rng.uniform() < 0.7)
        sense = 1 if rng.uniform() < 0.5 else -1
        out.append(Request(len(out), t, (nz, ny, nx), steps, fp32, sense,
                           int(rng.integers(0, 2 ** 31))))
    return out


def random_smooth(seed: int, shape, bc=BC_PERIODIC, cmax=0.15, hvar=0.2,
                  divergence_free=False) -> Fields:
    """Generic seeded test case: smooth positive psi, smooth variable h in
    [1-hvar, 1+hvar], face Courant numbers of magnitude <= cmax (random
    smooth, or divergence-free from a streamfunction quantised to 2**-16)."""
    rng = _rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")

    def smooth(n_modes, amp):
        f = np.zeros(shape)
        for _ in range(n_modes):
            k = rng.integers(0, 3, 3)
            ph = rng.uniform(0, 2 * math.pi)
            f += amp * np.sin(2 * math.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz)
                              + ph) / n_modes
        return f

    psi = 1.0 + 0.5 * smooth(3, 1.0) + 0.05 * rng.uniform(size=shape)
    h = 1.0 + smooth(2, hvar)
    if divergence_free:
        s = rng.normal(size=(nz, ny + 1, nx + 1))
        if bc == BC_PERIODIC:
            s[:, -1, :] = s[:, 0, :]
            s[:, :, -1] = s[:, :, 0]
        u1 = s[:, 1:, :] - s[:, :-1, :]
        u2 = -(s[:, :, 1:] - s[:, :, :-1])
        scale = cmax / max(np.abs(u1).max(), np.abs(u2).max(), 1e-300)
        q = 2.0 ** -16
        s = np.round(s * scale / q) * q
        u1 = s[:, 1:, :] - s[:, :-1, :]
        u2 = -(s[:, :, 1:] - s[:, :, :-1])
        u3 = np.zeros((nz + 1, ny, nx))
    else:
        u1 = rng.uniform(-cmax, cmax, (nz, ny, nx + 1))
        u2 = rng.uniform(-cmax, cmax, (nz, ny + 1, nx))
        u3 = rng.uniform(-cmax, cmax, (nz + 1, ny, nx))
        if bc == BC_PERIODIC:
            u1[:, :, -1] = u1[:, :, 0]
            u2[:, -1, :] = u2[:, 0, :]
            u3[-1, :, :] = u3[0, :, :]
    return Fields(np.ascontiguousarray(psi), np.ascontiguousarray(u1),
                  np.ascontiguousarray(u2), np.ascontiguousarray(u3),
                  np.ascontiguousarray(h), bc)
