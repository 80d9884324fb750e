"""Seeded synthetic calcium-imaging stacks.

This module only draws inputs: smooth backgrounds, Gaussian "somata", planted
integer translations, Gaussian or Poisson noise.  It holds none of the
alignment arithmetic and imports neither the oracle nor the library, so both
sides of every parity test can take their inputs from it.

Every frame has its own seed, ``SeedSequence([seed, family, stack, frame])``;
the scene (background and blobs) uses frame id 2**20 and the shift path 2**20+1.
A frame can therefore be regenerated on its own, in any order, in parallel.

Two families stand in for the paper's private videos (same shapes as its
timing table, structure of two-photon calcium imaging):

* ``BlobScene`` float32: noise-free base image as template, frames are the base
  rolled by a planted shift plus Gaussian noise.
* ``PoissonScene`` uint16: photon counts with per-frame blob flicker and a
  random-walk drift with jumps; the template is frame 0.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass

import numpy as np

SCENE_ID = 2 ** 20
PATH_ID = 2 ** 20 + 1
FAMILY_F32 = 1
FAMILY_U16 = 2


def _rng(*ids) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(v) for v in ids])))


def _background(rng, m: int, n: int) -> np.ndarray:
    p1, p2 = rng.uniform(0.0, 2 * np.pi, size=2)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    return 1.0 + 0.5 * np.cos(2 * np.pi * i / m + p1) * np.cos(2 * np.pi * j / n + p2)


def _blob_factors(rng, m: int, n: int, k: int, sig_lo: float, sig_hi: float):
    """Separable Gaussian blobs: returns row factors (m,k), column factors (n,k), amplitudes (k,)."""
    ci = rng.uniform(0, m, size=k)
    cj = rng.uniform(0, n, size=k)
    sig = rng.uniform(sig_lo, sig_hi, size=k)
    amp = rng.uniform(0.5, 2.0, size=k)
    i = np.arange(m)[:, None]
    j = np.arange(n)[:, None]
    gr = np.exp(-0.5 * ((i - ci[None, :]) / sig[None, :]) ** 2)
    gc = np.exp(-0.5 * ((j - cj[None, :]) / sig[None, :]) ** 2)
    return gr, gc, amp


@dataclass
class BlobScene:
    """float32 Gaussian blobs on a smooth cosine background, Gaussian noise."""
    m: int
    n: int
    nblobs: int
    max_shift: int
    noise_sigma: float
    seed: int = 0
    stack: int = 0
    sig_lo: float = 2.0
    sig_hi: float = 4.0

    def __post_init__(self):
        rng = _rng(self.seed, FAMILY_F32, self.stack, SCENE_ID)
        bg = _background(rng, self.m, self.n)
        gr, gc, amp = _blob_factors(rng, self.m, self.n, self.nblobs, self.sig_lo, self.sig_hi)
        self.base = (bg + (gr * amp[None, :]) @ gc.T).astype(np.float32)

    @property
    def template(self) -> np.ndarray:
        return self.base

    def shift(self, k: int):
        rng = _rng(self.seed, FAMILY_F32, self.stack, k)
        s, t = rng.integers(-self.max_shift, self.max_shift + 1, size=2)
        return int(s), int(t)

    def frame(self, k: int) -> np.ndarray:
        rng = _rng(self.seed, FAMILY_F32, self.stack, k)
        s, t = rng.integers(-self.max_shift, self.max_shift + 1, size=2)
        noise = rng.standard_normal((self.m, self.n)) * self.noise_sigma
        return (np.roll(self.base, (int(s), int(t)), axis=(0, 1)) + noise).astype(np.float32)

    def frames(self, k0: int, k1: int) -> np.ndarray:
        return np.stack([self.frame(k) for k in range(k0, k1)]) if k1 > k0 else \
            np.zeros((0, self.m, self.n), np.float32)

    def shifts(self, k0: int, k1: int) -> np.ndarray:
        return np.array([self.shift(k) for k in range(k0, k1)], np.int32).reshape(-1, 2)


@dataclass
class PoissonScene:
    """uint16 photon counts: mean 200, blob flicker, random-walk drift plus jumps."""
    m: int
    n: int
    T: int
    seed: int = 0
    stack: int = 0
    mean: float = 200.0
    max_shift: int = 50
    jump_prob: float = 0.01
    flicker: float = 0.2
    blobs_per_512sq: int = 300

    def __post_init__(self):
        rng = _rng(self.seed, FAMILY_U16, self.stack, SCENE_ID)
        k = max(1, int(round(self.blobs_per_512sq * self.m * self.n / 512.0 ** 2)))
        self.bg = _background(rng, self.m, self.n)
        self.gr, self.gc, self.amp = _blob_factors(rng, self.m, self.n, k, 3.0, 5.0)
        lam0 = self.bg + (self.gr * self.amp[None, :]) @ self.gc.T
        self.scale = self.mean / float(lam0.mean())
        # shift path: S_0 = (0,0); unit random-walk steps, rare uniform jumps, clamped
        prng = _rng(self.seed, FAMILY_U16, self.stack, PATH_ID)
        path = np.zeros((max(self.T, 1), 2), np.int64)
        L = self.max_shift
        for f in range(1, self.T):
            step = np.rint(prng.standard_normal(2)).astype(np.int64)
            cur = path[f - 1] + step
            if prng.uniform() < self.jump_prob:
                cur = prng.integers(-L, L + 1, size=2)
            path[f] = np.clip(cur, -L, L)
        self.path = path[: self.T].astype(np.int32)

    def shift(self, k: int):
        return int(self.path[k, 0]), int(self.path[k, 1])

    def shifts(self, k0: int, k1: int) -> np.ndarray:
        return self.path[k0:k1].copy()

    def frame(self, k: int) -> np.ndarray:
        rng = _rng(self.seed, FAMILY_U16, self.stack, k)
        z = rng.standard_normal(self.amp.shape[0])
        amp = self.amp * np.exp(self.flicker * z)
        lam = (self.bg + (self.gr * amp[None, :]) @ self.gc.T) * self.scale
        lam = np.roll(lam, self.shift(k), axis=(0, 1))
        x = rng.poisson(lam)
        return np.clip(x, 0, 65535).astype(np.uint16)

    @property
    def template(self) -> np.ndarray:
        return self.frame(0)

    def frames(self, k0: int, k1: int, workers: int = 1) -> np.ndarray:
        out = np.empty((max(0, k1 - k0), self.m, self.n), np.uint16)
        if workers <= 1 or k1 - k0 < 64:
            for k in range(k0, k1):
                out[k - k0] = self.frame(k)
            return out
        bounds = np.linspace(k0, k1, workers * 4 + 1).astype(int)
        jobs = [(self, int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
        with ProcessPoolExecutor(max_workers=workers, initializer=_one_blas_thread) as ex:
            for (_, a, b), chunk in zip(jobs, ex.map(_poisson_chunk, jobs)):
                out[a - k0:b - k0] = chunk
        return out


def _one_blas_thread():
    # each worker process draws frames serially; a multi-threaded BLAS in every
    # worker would oversubscribe the cores
    try:
        import threadpoolctl
        global _TP_LIMIT
        _TP_LIMIT = threadpoolctl.threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        pass


def _poisson_chunk(job):
    scene, a, b = job
    return np.stack([scene.frame(k) for k in range(a, b)])


def default_workers() -> int:
    """Worker processes for stack generation: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# ---------------------------------------------------------------------------
# Named workloads (sizes of the evaluation; each is synthetic)
# ---------------------------------------------------------------------------

def blobs128_f32(seed: int = 0) -> BlobScene:
    """100 frames of 128x128 float32, ~50 blobs, shifts U{-8..8}^2, noise 0.1; no downsampling, w=10."""
    return BlobScene(128, 128, nblobs=50, max_shift=8, noise_sigma=0.1, seed=seed)


def lowsnr256_f32(seed: int = 0) -> BlobScene:
    """256x256 float32 at low SNR (noise 0.625 = half the mean amplitude), shifts up to 60, w=64."""
    return BlobScene(256, 256, nblobs=200, max_shift=60, noise_sigma=0.625, seed=seed)


def poisson512_u16(T: int = 2000, seed: int = 0) -> PoissonScene:
    """512x512 uint16 Poisson photon counts (mean 200), drift + jumps up to 50 px; ds to 256^2, w=32."""
    return PoissonScene(512, 512, T, seed=seed)


WORKLOADS = {
    "blobs128_f32_w10": dict(T=100, m=128, n=128, w=10, downsample=False, dtype="f32"),
    "poisson512_u16_ds_w32": dict(T=2000, m=512, n=512, w=32, downsample=True, dtype="u16"),
    "lowsnr256_f32_w64": dict(T=10000, m=256, n=256, w=64, downsample=False, dtype="f32"),
}


def mixed_stacks(nstacks: int = 64, seed: int = 0, max_len: int = 3000, min_len: int = 50):
    """Uneven batch: per stack a frame size from {128^2, 256^2, 512^2, 512x796}, a length
    U{min_len..max_len}, a window from {8,16,32,48}; downsampled iff a side exceeds 256.
    Planted shifts are clamped so that the truth stays inside the searched window."""
    rng = _rng(seed, 3, 0, SCENE_ID)
    sizes = [(128, 128), (256, 256), (512, 512), (512, 796)]
    out = []
    for k in range(nstacks):
        m, n = sizes[int(rng.integers(0, 4))]
        T = int(rng.integers(min_len, max_len + 1))
        w = int(rng.choice([8, 16, 32, 48]))
        ds = m > 256 or n > 256
        mg, ng = (m // 2, n // 2) if ds else (m, n)
        w = min(w, mg, ng)
        lim = min(50, int(0.8 * (w - 1)) * (2 if ds else 1))
        sc = PoissonScene(m, n, T, seed=seed, stack=k + 1, max_shift=max(lim, 0))
        out.append(dict(scene=sc, T=T, m=m, n=n, w=w, downsample=ds))
    return out


FAMILY_TIES = 4


def row_periodic(m: int, n: int, T: int, dtype: str = "u16", max_shift: int = 4,
                 noisy_every: int = 0, seed: int = 0):
    """A template whose rows repeat with period two (two random rows, uint16 counts
    around 200 or float32 around 1) and frames that are exact rolls of it by
    planted shifts (|S|, |T| <= max_shift).  Every ``noisy_every``-th frame
    (0: none) also gets Poisson (uint16) or Gaussian (float32, sigma 0.1) noise.
    Many shifts then score exactly alike on the noise-free frames: the
    degenerate case of the search's ties.  Returns (template, frames, shifts)."""
    rng = _rng(seed, FAMILY_TIES, 0, SCENE_ID)
    if dtype == "u16":
        rows = rng.integers(100, 300, size=(2, n)).astype(np.float64)
    else:
        rows = rng.uniform(0.5, 1.5, size=(2, n))
    base = rows[np.arange(m) % 2]
    shifts = rng.integers(-max_shift, max_shift + 1, size=(T, 2)).astype(np.int32)
    frames = np.empty((T, m, n), np.uint16 if dtype == "u16" else np.float32)
    for k in range(T):
        a = np.roll(base, (int(shifts[k, 0]), int(shifts[k, 1])), axis=(0, 1))
        if noisy_every and k % noisy_every == noisy_every - 1:
            fr = _rng(seed, FAMILY_TIES, 0, k)
            a = fr.poisson(a).astype(np.float64) if dtype == "u16" else \
                a + fr.normal(0.0, 0.1, size=a.shape)
        frames[k] = a
    tmpl = base.astype(np.uint16 if dtype == "u16" else np.float32)
    return tmpl, frames, shifts
