"""Seeded synthetic workloads for the CLOMP hot path.

This module only draws inputs; it holds none of the method's arithmetic and is
shared by the tests, the smoke check and the benchmark.  Storage convention:
a dictionary is returned atom-major, `At` of shape (n, lda) with row j holding
column a_j of the m x n matrix A (i.e. A stored column-major with leading
dimension lda >= m; entries [m:lda) of each row are zero padding).  The math
view is A = At[:, :m].T.

The paper's workloads are datasets that are not available here (real 1-D
ECG/EEG/WSN records and eight image sets).  The generators below stand in for
them with the paper's shapes: Gaussian measurement matrices A = M D, which for
an orthonormal DCT D and i.i.d. Gaussian M is again i.i.d. Gaussian (Results,
"Evaluation with synthetic 1D data"; Methods, Eq. (1)); DCT-domain sparse
coefficients with dominant low frequencies; columns of an image sharing one A
(Eq. (3)); an image flattened to one long signal; sampling rates 0.1 to 0.5.

Seeds: instance i of workload c draws from numpy PCG64 seeded with
[2501, 11592, c, i] (plus a sub-index for the image batch).  Device-side draws
(the multi-gigabyte matrices) use a torch.Generator seeded from the same tuple.
"""

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = (2501, 11592)


def rng_for(cfg, i, sub=0):
    return np.random.default_rng([SEED_BASE[0], SEED_BASE[1], cfg, i, sub])


def torch_seed_for(cfg, i, sub=0):
    return (SEED_BASE[0] * 1_000_003 + SEED_BASE[1] * 10_007 + cfg * 101
            + i * 7 + sub) % (2 ** 63 - 1)


def pad_lda(m, elem_bytes=4, align_bytes=128):
    """Leading dimension rounded up so each atom starts on an aligned boundary."""
    q = max(1, align_bytes // elem_bytes)
    return ((m + q - 1) // q) * q


@dataclass
class Signal:
    At: np.ndarray        # (n, lda) atom-major storage of A (float32 or float64)
    m: int
    y: np.ndarray         # (m,) float32 measurements
    k: int
    support: np.ndarray   # true support (sorted)
    s: np.ndarray         # (n,) true coefficients (float64)

    @property
    def n(self):
        return self.At.shape[0]

    @property
    def A(self):
        """m x n float64 view of the stored values (for the oracle)."""
        return self.At[:, :self.m].T.astype(np.float64)


def _pack(At_nm, lda, dtype):
    n, m = At_nm.shape
    out = np.zeros((n, lda), dtype=dtype)
    out[:, :m] = At_nm
    return out


# ---------------------------------------------------------------- workload 1
def single_small(i, n=256, m=64, k=8, lda=None, dtype=np.float32):
    """n=256, m=64, k=8: A iid N(0, 1/m) drawn in float64; support uniform
    without replacement; non-zeros N(0,1); noiseless y = A s.  The stored A is
    the float64 draw rounded to `dtype`; y is computed from the stored A."""
    g = rng_for(1, i)
    A64 = g.standard_normal((m, n)) / math.sqrt(m)
    supp = np.sort(g.choice(n, size=k, replace=False))
    s = np.zeros(n)
    s[supp] = g.standard_normal(k)
    lda = lda or pad_lda(m)
    At = _pack(A64.T, lda, dtype)
    y = (At[:, :m].T.astype(np.float64) @ s).astype(np.float32)
    return Signal(At, m, y, k, supp, s)


# ---------------------------------------------------------------- workload 2
def single_large(i=0, n=16384, m=4096, k=256, noise_var=1e-4, lda=None):
    """n=16384, m=4096, k=256: A iid N(0, 1/m) float32; non-zeros
    +-(1 + |N(0,1)|) on a uniform support; y = A s + N(0, noise_var)."""
    g = rng_for(2, i)
    At = g.standard_normal((n, m), dtype=np.float32)
    At *= np.float32(1.0 / math.sqrt(m))
    lda = lda or pad_lda(m)
    if lda != m:
        At = _pack(At, lda, np.float32)
    supp = np.sort(g.choice(n, size=k, replace=False))
    s = np.zeros(n)
    s[supp] = g.choice([-1.0, 1.0], size=k) * (1.0 + np.abs(g.standard_normal(k)))
    noise = g.normal(0.0, math.sqrt(noise_var), size=m)
    y = (At[:, :m].T.astype(np.float64)[:, supp] @ s[supp] + noise).astype(np.float32)
    return Signal(np.ascontiguousarray(At), m, y, k, supp, s)


# ---------------------------------------------------------------- workload 3
IMAGE_SR = (0.1, 0.3, 0.5)
IMAGE_M = {0.1: 26, 0.3: 77, 0.5: 128}


def power_law_coeffs(g, n, k, alpha=1.5):
    """k positions uniform without replacement; magnitudes i^-alpha (i=1..k)
    assigned in ascending position order (low frequencies dominate); random
    signs."""
    supp = np.sort(g.choice(n, size=k, replace=False))
    mags = np.arange(1, k + 1, dtype=np.float64) ** (-alpha)
    s = np.zeros(n)
    s[supp] = mags * g.choice([-1.0, 1.0], size=k)
    return supp, s


@dataclass
class SharedBatch:
    At: np.ndarray        # (n, lda) float32, shared by every column
    m: int
    Y: np.ndarray         # (a, m) float32: row c is the measurement of signal c
    k: int
    supports: list
    S: np.ndarray         # (a, n) true coefficients

    @property
    def n(self):
        return self.At.shape[0]

    @property
    def A(self):
        return self.At[:, :self.m].T.astype(np.float64)


def image_batch(sr=0.3, n=256, a=256, k=32, lda=None):
    """Columns of a synthetic n x a image, each an n-long DCT-domain signal with
    power-law coefficients |c_i| ~ i^-1.5 truncated to k; one shared Gaussian A
    at sampling rate sr (m = 26 / 77 / 128 for sr = 0.1 / 0.3 / 0.5); Y = A S."""
    m = IMAGE_M[sr]
    g = rng_for(3, IMAGE_SR.index(sr))
    At = (g.standard_normal((n, m)) / math.sqrt(m)).astype(np.float32)
    lda = lda or pad_lda(m)
    At = _pack(At, lda, np.float32)
    A64 = At[:, :m].T.astype(np.float64)
    sup, S = [], np.zeros((a, n))
    for c in range(a):
        sp, s = power_law_coeffs(g, n, k)
        sup.append(sp)
        S[c] = s
    Y = (S @ A64.T).astype(np.float32)
    return SharedBatch(At, m, Y, k, sup, S)


IMAGE4K_SR = (0.1, 0.3, 0.5)


def image4k_batch(sr=0.3, n=2160, a=3840, k=108, lda=None):
    """A 4K-scale image (3840 x 2160) as a columns batch: 3840 signals of n =
    2160 rows sharing one Gaussian A with m = round(sr * n) (216 / 648 / 1080),
    each column k-sparse with power-law coefficients |c_i| ~ i^-1.5 (k = 5% of
    n, the low sparse rate of 4K images); Y = A S."""
    m = int(round(sr * n))
    g = rng_for(6, IMAGE4K_SR.index(sr))
    At = (g.standard_normal((n, m)) / math.sqrt(m)).astype(np.float32)
    lda = lda or pad_lda(m)
    At = _pack(At, lda, np.float32)
    A64 = At[:, :m].T.astype(np.float64)
    sup, S = [], np.zeros((a, n))
    for c in range(a):
        sp, s = power_law_coeffs(g, n, k)
        sup.append(sp)
        S[c] = s
    Y = (S @ A64.T).astype(np.float32)
    return SharedBatch(At, m, Y, k, sup, S)


# ---------------------------------------------------------------- workload 4
@dataclass
class UnevenSpec:
    n: int
    m: int
    k: int


def uneven_specs(count=4096, n_lo=512, n_hi=8192):
    """Sizes of the uneven batch: n log-uniform in [n_lo, n_hi], m/n uniform in
    [0.1, 0.5], k uniform integer in [ceil(n/64), floor(n/16)]."""
    specs = []
    for i in range(count):
        g = rng_for(4, i)
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        m = max(1, int(round(n * g.uniform(0.1, 0.5))))
        k = int(g.integers(math.ceil(n / 64), math.floor(n / 16) + 1))
        specs.append(UnevenSpec(n, m, k))
    return specs


def uneven_instance_host(i, spec):
    """One instance of the uneven batch drawn on the host: A iid N(0, 1/m) as a
    float32 master; non-zeros N(0,1) on a uniform support; noiseless y."""
    g = rng_for(4, i, 1)
    n, m, k = spec.n, spec.m, spec.k
    lda = pad_lda(m)
    At = _pack((g.standard_normal((n, m)) / math.sqrt(m)).astype(np.float32),
               lda, np.float32)
    supp = np.sort(g.choice(n, size=k, replace=False))
    s = np.zeros(n)
    s[supp] = g.standard_normal(k)
    y = (At[:, :m].T.astype(np.float64)[:, supp] @ s[supp]).astype(np.float32)
    return Signal(At, m, y, k, supp, s)


# ---------------------------------------------------------------- workload 5
FLAT_N, FLAT_M, FLAT_K = 65536, 19661, 2048


def flat_image_coeffs(n=FLAT_N, k=FLAT_K):
    """Power-law-compressible coefficients of a flattened 256 x 256 image,
    truncated to k non-zeros."""
    g = rng_for(5, 0)
    return power_law_coeffs(g, n, k)


def device_gaussian_atoms(n, m, lda, seed, device, chunk_atoms=4096):
    """Draw A iid N(0, 1/m) directly on `device` as an (n, lda) float32 tensor
    (zero padding beyond m), from a seeded torch.Generator."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    At = torch.zeros((n, lda), dtype=torch.float32, device=device)
    scale = 1.0 / math.sqrt(m)
    for j0 in range(0, n, chunk_atoms):
        j1 = min(n, j0 + chunk_atoms)
        blk = torch.randn((j1 - j0, m), generator=gen, device=device,
                          dtype=torch.float32)
        At[j0:j1, :m] = blk * scale
    return At


# --------------------------------------------------- host draws with goldens
def measurements(At, m, supp, s_supp):
    """y = A_S s_S for a noiseless instance: the float64 products of the stored
    columns summed by numpy's fixed-order reduction (no BLAS, so the value does
    not depend on the host's thread count), rounded to float32."""
    AS = np.asarray(At[np.asarray(supp), :m], dtype=np.float64)
    return (AS * np.asarray(s_supp, dtype=np.float64)[:, None]).sum(axis=0).astype(np.float32)


def bf16_values(At32):
    """The bfloat16 storage of a float32 array (round to nearest even), returned
    as the float32 array of the stored values."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(At32)).to(torch.bfloat16).to(
        torch.float32).numpy()


def uneven_golden_indices(specs, count=16):
    """Stratified sample of the uneven batch: the instances at the centres of
    `count` equal strata of the batch sorted by n, the last stratum replaced by
    the largest n.  These are drawn on the host so the oracle can regenerate
    them."""
    order = np.argsort([sp.n for sp in specs], kind="stable")
    N = len(order)
    pos = [int((q + 0.5) * N / count) for q in range(count - 1)] + [N - 1]
    return [int(order[p]) for p in pos]


def uneven_instance_golden(i, spec):
    """Instance i of the uneven batch as the host draws it (the stratified
    sample): A iid N(0, 1/m) float32 master (lda a multiple of 32), N(0, 1)
    non-zeros on a uniform support, noiseless y = A s (fixed-order sum)."""
    g = rng_for(4, i, 3)
    n, m, k = spec.n, spec.m, spec.k
    blk = g.standard_normal((n, m), dtype=np.float32)
    blk *= np.float32(1.0 / math.sqrt(m))
    At = _pack(blk, pad_lda(m, 4), np.float32)
    supp = np.sort(g.choice(n, size=k, replace=False))
    s = np.zeros(n)
    s[supp] = g.standard_normal(k)
    return Signal(At, m, measurements(At, m, supp, s[supp]), k, supp, s)


FLAT_CHUNK = 4096


def flat_image_host(n=FLAT_N, m=FLAT_M, k=FLAT_K, workers=None):
    """The flattened 256 x 256 image drawn on the host: A iid N(0, 1/m) as an
    (n, lda) float32 array, atoms j0 .. j0+4095 drawn from their own PCG64
    stream (so several threads can fill it and the values do not depend on
    their number); power-law coefficients truncated to k; noiseless y = A s
    (fixed-order sum).  Returns (At, y, supp, s)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    lda = pad_lda(m, 4)
    At = np.zeros((n, lda), dtype=np.float32)
    scale = np.float32(1.0 / math.sqrt(m))

    def fill(c):
        j0 = c * FLAT_CHUNK
        j1 = min(n, j0 + FLAT_CHUNK)
        blk = rng_for(5, 0, 100 + c).standard_normal((j1 - j0, m), dtype=np.float32)
        blk *= scale
        At[j0:j1, :m] = blk

    nchunk = (n + FLAT_CHUNK - 1) // FLAT_CHUNK
    with ThreadPoolExecutor(max_workers=workers or min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(nchunk)))
    supp, s = flat_image_coeffs(n, k)
    return At, measurements(At, m, supp, s[supp]), supp, s


def fingerprint(a):
    """sha256 of an array's bytes (inputs of a stored oracle result)."""
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ------------------------------------------------------------ device batches
def uneven_batch_device(count=4096, device="cuda", golden=True):
    """The uneven batch drawn on the device: per instance an FP32 master
    (lda rounded to 32) and its bfloat16 copy (lda rounded to 64), packed in two
    flat buffers; y = A s computed from the master in float64 on the device.
    With golden=True the stratified sample (uneven_golden_indices) is drawn on
    the host instead (uneven_instance_golden, bfloat16 rounding on the host)
    and uploaded.  Returns (specs, items, supports, coefficient dicts)."""
    import torch
    specs = uneven_specs(count)
    gold = set(uneven_golden_indices(specs)) if golden and count == 4096 else set()
    lda32 = [pad_lda(sp.m, 4) for sp in specs]
    lda16 = [pad_lda(sp.m, 2) for sp in specs]
    tot32 = sum(sp.n * l for sp, l in zip(specs, lda32))
    tot16 = sum(sp.n * l for sp, l in zip(specs, lda16))
    buf32 = torch.empty(tot32, dtype=torch.float32, device=device)
    buf16 = torch.empty(tot16, dtype=torch.bfloat16, device=device)
    items, supports, coefs = [], [], []
    o32 = o16 = 0
    for i, sp in enumerate(specs):
        n, m, k = sp.n, sp.m, sp.k
        Am = buf32[o32:o32 + n * lda32[i]].view(n, lda32[i])
        Ab = buf16[o16:o16 + n * lda16[i]].view(n, lda16[i])
        o32 += n * lda32[i]
        o16 += n * lda16[i]
        if i in gold:
            sig = uneven_instance_golden(i, sp)
            Am.copy_(torch.from_numpy(sig.At))
            Ab.zero_()
            Ab[:, :m] = torch.from_numpy(bf16_values(sig.At[:, :m])).to(device).to(torch.bfloat16)
            items.append(dict(At=Ab, m=m, y=torch.from_numpy(sig.y).to(device), k=k,
                              At_master=Am))
            supports.append(sig.support)
            coefs.append(sig.s[sig.support])
            continue
        gen = torch.Generator(device=device)
        gen.manual_seed(torch_seed_for(4, i))
        Am.zero_()
        Am[:, :m] = torch.randn((n, m), generator=gen, device=device) * (1.0 / math.sqrt(m))
        Ab.zero_()
        Ab[:, :m] = Am[:, :m].to(torch.bfloat16)
        g = rng_for(4, i, 2)
        supp = np.sort(g.choice(n, size=k, replace=False))
        s = g.standard_normal(k)
        st = torch.as_tensor(s, device=device)
        idx = torch.as_tensor(supp, device=device)
        y = (Am[idx, :m].double().T @ st).float().contiguous()
        items.append(dict(At=Ab, m=m, y=y, k=k, At_master=Am))
        supports.append(supp)
        coefs.append(s)
    return specs, items, supports, coefs


def flat_image_device(device="cuda", host=None, m=FLAT_M):
    """The flattened 256 x 256 image on the device: the host draw of
    flat_image_host (or `host`, its result) uploaded as the FP32 master, and
    its bfloat16 copy rounded on the host.  Returns (Am, Ab, y, supp, s)."""
    import torch
    At, y, supp, s = host if host is not None else flat_image_host(m=m)
    n = At.shape[0]
    Am = torch.from_numpy(At).to(device)
    Ab = torch.zeros((n, pad_lda(m, 2)), dtype=torch.bfloat16, device=device)
    for j0 in range(0, n, FLAT_CHUNK):
        j1 = min(n, j0 + FLAT_CHUNK)
        Ab[j0:j1, :m] = torch.from_numpy(At[j0:j1, :m]).to(torch.bfloat16).to(device)
    return Am, Ab, torch.from_numpy(y).to(device), supp, s
