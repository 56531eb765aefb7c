"""Seeded synthetic exposure stacks: the inputs both the HIP path and the oracle consume.

This module holds none of the alignment method's arithmetic (no gray conversion,
no pyramid, no median, no bitmaps, no search).  It only draws scenes and
exposures, so that the two sides under comparison are fed the same bytes.

The paper measures on its own 3.7 MP photo sets of 5 exposures (Section IV,
Fig. 3), which are not available here.  These generators stand in for them
with the same structure: 8-bit interleaved RGB exposures of one static scene,
2-stop spacing, 2-7 images per stack (Sections III-B and IV), each exposure
translated by an integer amount as a hand-held camera would.

Scene model (all arithmetic in float64):
  * Radiance per channel c: a sum of isotropic Gaussian blobs plus noise,
        Rad_c(x, y) = sum_b a_{b,c} exp(-((x-cx_b)^2 + (y-cy_b)^2) / (2 s_b^2)) + n_c(x, y)
    with centres uniform over the image, s_b ~ U[5, 60] px, a_{b,c} ~ U[0.1, 1]
    (three independent draws per blob) and n_c ~ Normal(0, sd=0.01) per pixel.
    Each blob is evaluated inside a +-4 s_b window.  The noise belongs to the
    scene, so every exposure of a stack shares it.
  * Exposure e with gain k: v = clip(k * 2^e * Rad, 0, 1), then the gamma-1/2.2
    8-bit code q = floor(255 v^(1/2.2) + 0.5).  q is computed exactly from its
    definition as the number of thresholds theta_j = ((j - 0.5)/255)^2.2,
    j = 1..255, that v reaches, so it does not depend on the host's pow().
  * Translation by t = (tx, ty) with edge replicate:
        mov[y][x] = src[clamp(y - ty)][clamp(x - tx)]
    An aligner that reports the shift to apply to the moving image must then
    answer -t.

Randomness comes from numpy's PCG64 (``numpy.random.default_rng(seed)``) in a
fixed draw order: centres x, centres y, sigmas, amplitudes, noise, then shifts.
"""

from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "THRESHOLDS",
    "radiance_field",
    "rect_field",
    "make_rect_pair",
    "expose",
    "translate",
    "saturation_gain",
    "make_pair",
    "make_stack",
    "Workload",
    "workload",
    "sha256",
]

# theta_j = ((j - 0.5) / 255)^2.2 for j = 1..255; code q >= j  <=>  v >= theta_j.
THRESHOLDS = np.array([math.pow((j - 0.5) / 255.0, 2.2) for j in range(1, 256)], dtype=np.float64)
# Bracket table: code q holds exactly when _BRACKET[q] <= v < _BRACKET[q + 1].
_BRACKET = np.concatenate(([-np.inf], THRESHOLDS, [np.inf]))
# Rows per chunk for the elementwise passes (keeps temporaries small; no effect on values).
_CHUNK = 64


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def radiance_field(width: int, height: int, n_blobs: int, rng: np.random.Generator) -> np.ndarray:
    """float64 radiance, shape (3, H, W), drawn as described in the module docstring."""
    W, H = int(width), int(height)
    cx = rng.uniform(0.0, W, n_blobs)
    cy = rng.uniform(0.0, H, n_blobs)
    sig = rng.uniform(5.0, 60.0, n_blobs)
    amp = rng.uniform(0.1, 1.0, (n_blobs, 3))
    rad = np.zeros((3, H, W), dtype=np.float64)
    for b in range(n_blobs):
        s = float(sig[b])
        x0 = max(0, math.ceil(cx[b] - 4.0 * s))
        x1 = min(W - 1, math.floor(cx[b] + 4.0 * s))
        y0 = max(0, math.ceil(cy[b] - 4.0 * s))
        y1 = min(H - 1, math.floor(cy[b] + 4.0 * s))
        if x0 > x1 or y0 > y1:
            continue
        inv = 1.0 / (2.0 * s * s)
        # Separable: exp(-(dx^2+dy^2)/2s^2) = exp(-dx^2/2s^2) * exp(-dy^2/2s^2).
        # math.exp keeps the values independent of numpy's SIMD dispatch.
        gx = np.array([math.exp(-((x - cx[b]) ** 2) * inv) for x in range(x0, x1 + 1)])
        gy = np.array([math.exp(-((y - cy[b]) ** 2) * inv) for y in range(y0, y1 + 1)])
        g = np.multiply.outer(gy, gx)
        for c in range(3):
            rad[c, y0:y1 + 1, x0:x1 + 1] += amp[b, c] * g
    # Noise is drawn channel by channel in row order; drawing it in row chunks
    # consumes the generator exactly as one (3, H, W) draw would.
    for c in range(3):
        for y in range(0, H, _CHUNK):
            y1 = min(H, y + _CHUNK)
            rad[c, y:y1] += rng.normal(0.0, 0.01, (y1 - y, W))
    return rad


def rect_field(width: int, height: int, n_rects: int, rng: np.random.Generator) -> np.ndarray:
    """float64 radiance (3, H, W) of overlapping axis-aligned rectangles plus noise.

    A sharp-edged scene for tests: a floor of 0.05, then n_rects rectangles with
    top-left corner uniform over the image, sides uniform in [4, W/3) and
    [4, H/3), and per-channel amplitude U[0, 0.6] added inside; then
    Normal(0, sd=0.01) noise per pixel, drawn channel by channel in row order.
    Blob fields are smooth, so a one-pixel shift moves few pixels across the
    median by more than the exclusion band; this scene gives every candidate
    shift a clearly different error.
    """
    W, H = int(width), int(height)
    rad = np.full((3, H, W), 0.05, dtype=np.float64)
    for _ in range(n_rects):
        x0 = int(rng.integers(0, W))
        y0 = int(rng.integers(0, H))
        w = int(rng.integers(4, max(5, W // 3)))
        h = int(rng.integers(4, max(5, H // 3)))
        a = rng.uniform(0.0, 0.6, 3)
        rad[:, y0:y0 + h, x0:x0 + w] += a[:, None, None]
    for c in range(3):
        for y in range(0, H, _CHUNK):
            y1 = min(H, y + _CHUNK)
            rad[c, y:y1] += rng.normal(0.0, 0.01, (y1 - y, W))
    return rad


def make_rect_pair(width, height, n_rects, seed, shift_range, evs=(0.0, -2.0)):
    """Like make_pair, on a rect_field scene.  Returns (ref, mov, (tx, ty))."""
    rng = np.random.default_rng(seed)
    rad = rect_field(width, height, n_rects, rng)
    tx, ty = (int(v) for v in rng.integers(-shift_range, shift_range + 1, 2))
    ref = expose(rad, evs[0])
    mov = translate(expose(rad, evs[1]), tx, ty)
    return ref, mov, (tx, ty)


def _quantise(v: np.ndarray) -> np.ndarray:
    """Exact gamma-1/2.2 8-bit code of v in [0, 1] (see module docstring)."""
    q = np.floor(255.0 * np.power(v.astype(np.float32), np.float32(1.0 / 2.2)) + 0.5)
    q = np.clip(q, 0, 255).astype(np.int64)
    # One correction step makes the float32 estimate exact (it is never off by more than one).
    q += (v >= _BRACKET[q + 1]).astype(np.int64)
    q -= (v < _BRACKET[q]).astype(np.int64)
    return q.astype(np.uint8)


def expose(rad: np.ndarray, ev: float, gain: float = 1.0) -> np.ndarray:
    """Interleaved RGB uint8 image (H, W, 3) of radiance ``rad`` (3, H, W) at exposure 2^ev."""
    scale = float(gain) * math.pow(2.0, ev)
    _, H, W = rad.shape
    out = np.empty((H, W, 3), dtype=np.uint8)
    for y in range(0, H, _CHUNK):
        y1 = min(H, y + _CHUNK)
        for c in range(3):
            v = np.clip(rad[c, y:y1] * scale, 0.0, 1.0)
            out[y:y1, :, c] = _quantise(v)
    return out


def translate(img: np.ndarray, tx: int, ty: int) -> np.ndarray:
    """Edge-replicate translation: out[y][x] = img[clamp(y - ty)][clamp(x - tx)]."""
    H, W = img.shape[:2]
    tx, ty = int(tx), int(ty)

    def shift_cols(dst, src):
        # dst[:, x] = src[:, clamp(x - tx)]
        xs, xe = min(max(tx, 0), W), max(min(W + tx, W), 0)
        if xs < xe:
            dst[:, xs:xe] = src[:, xs - tx:xe - tx]
            dst[:, :xs] = src[:, :1]
            dst[:, xe:] = src[:, W - 1:W]
        else:
            dst[:] = src[:, :1] if tx > 0 else src[:, W - 1:W]

    out = np.empty_like(img)
    ys, ye = min(max(ty, 0), H), max(min(H + ty, H), 0)
    if ys < ye:
        shift_cols(out[ys:ye], img[ys - ty:ye - ty])
        out[:ys] = out[ys]
        out[ye:] = out[ye - 1]
    else:
        shift_cols(out[:1], img[:1] if ty > 0 else img[H - 1:H])
        out[1:] = out[0]
    return out


def saturation_gain(rad: np.ndarray, evs, frac: float) -> float:
    """Gain k at which ``frac`` of the pixels pooled over the exposures saturate.

    A pixel saturates when any channel codes to 255, i.e. when
    k 2^e max_c Rad_c >= theta_255.  With the pooled set S = {2^e max_c Rad_c}
    over all pixels and exposures and V its K-th largest element,
    K = round(frac |S|), the gain is k = theta_255 / V.  S is never
    materialised: scaling by 2^e is exact, so counts come from one sorted copy.
    """
    s = np.sort(rad.max(axis=0), axis=None)
    n = s.size
    scales = [math.pow(2.0, e) for e in evs]
    K = max(1, int(round(frac * n * len(scales))))

    def count_ge(v: float) -> int:
        return sum(n - int(np.searchsorted(s, v / sc, side="left")) for sc in scales)

    best = -math.inf
    for sc in scales:
        # Largest index i with count_ge(s[i] * sc) >= K (count_ge decreases with i).
        lo, hi = -1, n - 1
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if count_ge(float(s[mid]) * sc) >= K:
                lo = mid
            else:
                hi = mid - 1
        if lo >= 0:
            best = max(best, float(s[lo]) * sc)
    return float(THRESHOLDS[-1] / best)


def make_pair(width, height, n_blobs, seed, shift_range, evs=(0.0, -2.0)):
    """Reference (exposure evs[0], unshifted) and moving (evs[1], translated) images.

    Returns (ref, mov, (tx, ty)); both images are (H, W, 3) uint8.
    """
    rng = np.random.default_rng(seed)
    rad = radiance_field(width, height, n_blobs, rng)
    tx, ty = (int(v) for v in rng.integers(-shift_range, shift_range + 1, 2))
    ref = expose(rad, evs[0])
    mov = translate(expose(rad, evs[1]), tx, ty)
    return ref, mov, (tx, ty)


def make_stack(width, height, n, n_blobs, seed, shift_range, sat_frac=None, evs=None):
    """Exposure stack of n images; the middle one (index n // 2) is the unshifted reference.

    Exposures default to 2^(i - n//2).  With ``sat_frac`` the gain is set so that
    that fraction of the pooled pixels saturate.  Returns (images, shifts, gain)
    where shifts[i] = (tx, ty) is the translation applied to image i.
    """
    rng = np.random.default_rng(seed)
    rad = radiance_field(width, height, n_blobs, rng)
    if evs is None:
        evs = [float(i - n // 2) for i in range(n)]
    gain = 1.0 if sat_frac is None else saturation_gain(rad, evs, sat_frac)
    ref = n // 2
    shifts = []
    for i in range(n):
        t = tuple(int(v) for v in rng.integers(-shift_range, shift_range + 1, 2))
        shifts.append((0, 0) if i == ref else t)
    images = []
    for i in range(n):
        img = expose(rad, evs[i], gain)
        tx, ty = shifts[i]
        if tx or ty:
            img = translate(img, tx, ty)
        images.append(img)
    return images, shifts, gain


@dataclass
class Workload:
    """One synthetic workload: a list of stacks (a pair is a stack of two)."""

    name: str
    width: int
    height: int
    levels: int
    stacks: list = field(default_factory=list)  # list of (images, shifts, ref_index)
    note: str = ""

    @property
    def megapixels(self) -> float:
        return sum(len(s[0]) for s in self.stacks) * self.width * self.height / 1e6


# Sizes (width, height, levels, blobs) of the uneven-batch workload.
BATCH_SIZES = ((640, 480, 5, 40), (1920, 1080, 6, 400), (4000, 3000, 7, 400), (6000, 4000, 7, 400))


def make_batch(n_pairs, seed, sizes=BATCH_SIZES, evs=(0.0, -2.0)):
    """A batch of 2-stop exposure pairs of uneven sizes.

    Each pair's size is drawn uniformly from ``sizes``; each size class has one
    radiance field (drawn in the order of ``sizes``) whose two exposures every
    pair of the class shares, the moving one translated by the pair's own
    shift t in [-2^(L-1), 2^(L-1)]^2 (edge replicate), drawn in pair order
    after the sizes.  Returns [(ref, mov, (tx, ty), levels), ...].
    """
    rng = np.random.default_rng(seed)
    cls = [int(c) for c in rng.integers(0, len(sizes), n_pairs)]
    shifts = []
    for c in cls:
        r = 1 << (sizes[c][2] - 1)
        shifts.append(tuple(int(v) for v in rng.integers(-r, r + 1, 2)))
    exposures = {}
    for c in sorted(set(cls)):
        W, H, _, blobs = sizes[c]
        rad = radiance_field(W, H, blobs, rng)
        exposures[c] = (expose(rad, evs[0]), expose(rad, evs[1]))
    out = []
    for c, (tx, ty) in zip(cls, shifts):
        ref, mov = exposures[c]
        out.append((ref, translate(mov, tx, ty), (tx, ty), sizes[c][2]))
    return out


def serve_levels(width: int, height: int) -> int:
    """Levels of a served request: min(7, 1 + floor(log2(min(W, H) / 32)))."""
    m = min(int(width), int(height))
    L = 1
    while L < 7 and (32 << L) <= m:
        L += 1
    return L


def make_serve_base(width, height, seed, n_exposures=9, n_blobs=400):
    """Base scene of the served workload: one radiance field, exposures 2^(e - n//2).

    Returns the list of (H, W, 3) uint8 exposures (index n//2 is 2^0).
    """
    rng = np.random.default_rng(seed)
    rad = radiance_field(width, height, n_blobs, rng)
    return [expose(rad, float(e - n_exposures // 2)) for e in range(n_exposures)]


def serve_requests(seed, rate, duration, base_width, base_height, n_exposures=9,
                   mp_range=(1.0, 48.0), n_range=(3, 9), aspect=1.5):
    """Poisson arrivals of exposure-stack requests cut from a base scene.

    Arrivals: exponential gaps with mean 1/rate until ``duration`` seconds.  Per
    request, in this order: n ~ U{n_range}; megapixels log-uniform over
    mp_range at the given aspect (W = round(sqrt(MP 1e6 aspect)), H =
    round(W / aspect), shrunk if needed to fit the base with margins); levels
    L = serve_levels(W, H), R = 2^(L-1); the reference crop's corner (x0, y0)
    uniform with every crop inside the base; offsets (dx, dy) in [-R, R]^2 for
    each non-reference image (the reference, index n//2, is at offset 0).
    Image i is exposure (n_exposures//2 + i - n//2) of the base cropped at
    (x0 + dx_i, y0 + dy_i); the shift that aligns it is (dx_i, dy_i).
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        lo, hi = math.log(mp_range[0]), math.log(mp_range[1])
        mp = math.exp(float(rng.uniform(lo, hi)))
        W = int(round(math.sqrt(mp * 1e6 * aspect)))
        H = int(round(W / aspect))
        L = serve_levels(W, H)
        R = 1 << (L - 1)
        W = min(W, base_width - 2 * R)
        H = min(H, base_height - 2 * R)
        L = serve_levels(W, H)
        R = 1 << (L - 1)
        x0 = int(rng.integers(R, base_width - W - R + 1))
        y0 = int(rng.integers(R, base_height - H - R + 1))
        offsets = []
        for i in range(n):
            d = tuple(int(v) for v in rng.integers(-R, R + 1, 2))
            offsets.append((0, 0) if i == n // 2 else d)
        exposures = [n_exposures // 2 + i - n // 2 for i in range(n)]
        out.append(dict(rid=len(out), arrival=t, n=n, width=W, height=H, levels=L, x0=x0, y0=y0,
                        offsets=offsets, exposures=exposures))
    return out


def serve_crop(base, req, i):
    """Image i of a served request as a view of the base exposures (any array type)."""
    dx, dy = req["offsets"][i]
    x, y = req["x0"] + dx, req["y0"] + dy
    return base[req["exposures"][i]][y:y + req["height"], x:x + req["width"]]


def workload(name: str) -> Workload:
    """The named synthetic workloads (sizes, seeds and ranges fixed here).

    pair_512x384     one pair 512x384,   40 blobs,  2^0 / 2^-2, t in [-20,20]^2, 5 levels, seed 1
    pair_4096x3072   one pair 4096x3072, 400 blobs, 2^0 / 2^-2, t in [-50,50]^2, 6 levels, seed 2
    stack7_6000x4000 seven 6000x4000 exposures 2^-3..2^3, middle reference unshifted,
                     t in [-100,100]^2 for the others, 5% pooled saturation, 400 blobs, 7 levels, seed 3
    """
    if name == "pair_512x384":
        ref, mov, t = make_pair(512, 384, 40, 1, 20)
        return Workload(name, 512, 384, 5, [([ref, mov], [(0, 0), t], 0)])
    if name == "pair_4096x3072":
        ref, mov, t = make_pair(4096, 3072, 400, 2, 50)
        return Workload(name, 4096, 3072, 6, [([ref, mov], [(0, 0), t], 0)])
    if name == "stack7_6000x4000":
        imgs, shifts, gain = make_stack(6000, 4000, 7, 400, 3, 100, sat_frac=0.05)
        return Workload(name, 6000, 4000, 7, [(imgs, shifts, 3)], note=f"gain={gain!r}")
    raise KeyError(name)
