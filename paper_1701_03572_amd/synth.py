"""Seeded synthetic UAV-like grayscale sequences with exact inter-frame ground truth.

This module is the input generator shared by the tests, the bench and the
oracle's callers. It holds none of the stabilizer's arithmetic: it renders a
continuous texture seen through a known chain of similarity cameras, so every
inter-frame transform is known exactly.

Rendering model. World coordinates are frame-0 pixel coordinates. Camera j is a
3x3 similarity A_j mapping world points to frame-j pixel coordinates (pixel
centres at integers, x = column, y = row), with A_0 = I. Frame j is

    F_j(y) = clip(round(T(A_j^{-1} y)), 0, 255)

where T is the texture, rasterised once on a world canvas at 1 px spacing and
read back with bicubic resampling (torch ``grid_sample``), so frames carry no
compounded resampling blur. The ground-truth pair transform S_j = A_{j+1} A_j^{-1}
maps frame-j points to frame-(j+1) points: the paper's src -> dst direction of
the motion model (Section 4, Eq. 7).

Workloads follow the paper's evaluation setting (UAV footage, Section 7) with
synthetic stand-ins, since the paper's videos are not available:

* ``tiny``  320x240,  60 frames, Gaussian-blob texture, i.i.d. similarity steps.
* ``vga``   640x480, 300 frames, blob texture, sinusoidal pan/yaw + jitter, 3
  independently moving 40x40 textured squares (outliers for the robust fit).
* ``hd``   1920x1080, 600 frames, fBm terrain, jitter x3, 120x120 movers.
* ``paper_*`` the paper's Table 2 shapes (frame counts and resolutions) with
  ``vga`` jitter, for context timings only.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch


@dataclasses.dataclass(frozen=True)
class SeqRecipe:
    name: str
    width: int
    height: int
    n_frames: int
    texture: str            # "blobs" or "fbm"
    motion: str             # "iid" (tiny) or "path" (sinusoid + jitter)
    jitter: float = 1.0     # multiplier on the "path" jitter
    n_movers: int = 0
    mover_size: int = 40
    seed: int = 1701


RECIPES = {
    "tiny": SeqRecipe("tiny", 320, 240, 60, "blobs", "iid", seed=1701),
    "vga": SeqRecipe("vga", 640, 480, 300, "blobs", "path", 1.0, 3, 40, seed=1702),
    "hd": SeqRecipe("hd", 1920, 1080, 600, "fbm", "path", 3.0, 3, 120, seed=1703),
    "hd720": SeqRecipe("hd720", 1280, 720, 300, "fbm", "path", 1.0, 3, 80, seed=1704),
    "uhd": SeqRecipe("uhd", 3840, 2160, 120, "fbm", "path", 1.0, 3, 160, seed=1706),
    "paper_forest": SeqRecipe("paper_forest", 320, 240, 1650, "blobs", "path", 1.0, 3, 40, seed=1801),
    "paper_ground": SeqRecipe("paper_ground", 640, 480, 966, "blobs", "path", 1.0, 3, 40, seed=1802),
    "paper_bird": SeqRecipe("paper_bird", 640, 360, 601, "blobs", "path", 1.0, 3, 40, seed=1803),
    "paper_girl": SeqRecipe("paper_girl", 640, 360, 446, "blobs", "path", 1.0, 3, 40, seed=1804),
}


# mixed-stream workload: resolution classes drawn uniformly, corner budgets U[100, 2000], levels
# clamp(1 + floor(log2(W / 80)), 3, 5), the 640x480 workload's jitter; stream s uses seed base * 1000 + s
MIXED_CLASSES = (("tiny", 320, 240), ("vga", 640, 480), ("hd720", 1280, 720), ("hd", 1920, 1080))


def mixed_streams(n_streams: int, n_frames: int, base_seed: int = 1705) -> list:
    """Per-stream (recipe, corner budget, levels) of a seeded mixed workload."""
    rng = np.random.default_rng(base_seed)
    out = []
    for s in range(n_streams):
        name, w, h = MIXED_CLASSES[int(rng.integers(0, len(MIXED_CLASSES)))]
        k = int(rng.integers(100, 2001))
        levels = int(min(5, max(3, 1 + math.floor(math.log2(w / 80)))))
        base = RECIPES[name]
        r = dataclasses.replace(base, name="%s_s%d" % (name, s), n_frames=max(n_frames, 2), motion="path", jitter=1.0,
                                seed=base_seed * 1000 + s)
        out.append((r, k, levels))
    return out


def recipe(name: str, **over) -> SeqRecipe:
    return dataclasses.replace(RECIPES[name], **over)


# ----------------------------------------------------------------------------------------------
# camera chain
# ----------------------------------------------------------------------------------------------

def similarity_about(angle: float, scale: float, tx: float, ty: float, cx: float, cy: float) -> np.ndarray:
    """3x3 similarity rotating by ``angle`` and scaling by ``scale`` about (cx, cy), then
    translating by (tx, ty)."""
    c, s = scale * math.cos(angle), scale * math.sin(angle)
    return np.array([[c, -s, cx - c * cx + s * cy + tx],
                     [s, c, cy - s * cx - c * cy + ty],
                     [0.0, 0.0, 1.0]])


def _cameras(r: SeqRecipe, rng: np.random.Generator) -> np.ndarray:
    """World->frame similarities A_j, shape (n, 3, 3), A_0 = I."""
    n, W, H = r.n_frames, r.width, r.height
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    A = np.zeros((n, 3, 3))
    if r.motion == "iid":
        # each frame is the previous one moved by an independent similarity
        A[0] = np.eye(3)
        for j in range(1, n):
            ang = math.radians(rng.normal(0.0, 0.5))
            sc = 1.0 + rng.normal(0.0, 0.005)
            tx = rng.normal(0.0, 3.0) + 1.0
            ty = rng.normal(0.0, 3.0)
            A[j] = similarity_about(ang, sc, tx, ty, cx, cy) @ A[j - 1]
        return A
    # smooth sinusoidal pan / yaw plus per-frame jitter of the absolute pose
    k = r.jitter
    amp_x, amp_y = 0.08 * W, 0.06 * H
    per_x, per_y, per_a = 240.0, 170.0, 300.0
    ph = rng.uniform(0, 2 * math.pi, size=3)
    j = np.arange(n, dtype=np.float64)
    px = amp_x * np.sin(2 * math.pi * j / per_x + ph[0]) + 0.5 * j
    py = amp_y * np.sin(2 * math.pi * j / per_y + ph[1])
    pa = math.radians(3.0) * np.sin(2 * math.pi * j / per_a + ph[2])
    jr = np.radians(rng.normal(0.0, 0.8 * k, size=n))
    jt = rng.normal(0.0, 5.0 * k, size=(n, 2))
    spikes = rng.random(n) < 0.05
    sdir = rng.uniform(0, 2 * math.pi, size=n)
    jt[spikes, 0] += 12.0 * k * np.cos(sdir[spikes])
    jt[spikes, 1] += 12.0 * k * np.sin(sdir[spikes])
    # the camera keeps its altitude and zoom: rotation and translation jitter only
    ang = pa + jr
    sc = np.ones(n)
    tx = px + jt[:, 0]
    ty = py + jt[:, 1]
    ang -= ang[0]
    sc /= sc[0]
    tx -= tx[0]
    ty -= ty[0]
    for i in range(n):
        A[i] = similarity_about(ang[i], sc[i], -tx[i], -ty[i], cx, cy)
    # re-base so that A_0 = I exactly
    inv0 = np.linalg.inv(A[0])
    for i in range(n):
        A[i] = A[i] @ inv0
    A[0] = np.eye(3)
    return A


# ----------------------------------------------------------------------------------------------
# textures on a world canvas
# ----------------------------------------------------------------------------------------------

def _blob_canvas(cw: int, ch: int, rng: np.random.Generator) -> np.ndarray:
    img = np.full((ch, cw), 20.0)
    n_blobs = max(1, int(round(200.0 * cw * ch / (320.0 * 240.0))))
    cxs = rng.uniform(0, cw, n_blobs)
    cys = rng.uniform(0, ch, n_blobs)
    sig = rng.uniform(2.0, 12.0, n_blobs)
    amp = rng.uniform(40.0, 200.0, n_blobs)
    for bx, by, s, a in zip(cxs, cys, sig, amp):
        rad = int(math.ceil(4 * s))
        x0, x1 = max(0, int(bx) - rad), min(cw, int(bx) + rad + 1)
        y0, y1 = max(0, int(by) - rad), min(ch, int(by) + rad + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1) - bx
        ys = np.arange(y0, y1) - by
        img[y0:y1, x0:x1] += a * np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2 * s * s))
    # band-limited noise: a seeded sum of plane waves with |f| <= 0.2 cycles/px
    yy, xx = np.mgrid[0:ch, 0:cw].astype(np.float64)
    noise = np.zeros_like(img)
    n_waves = 48
    for _ in range(n_waves):
        f = rng.uniform(0.02, 0.2)
        th = rng.uniform(0, 2 * math.pi)
        phs = rng.uniform(0, 2 * math.pi)
        noise += np.cos(2 * math.pi * f * (math.cos(th) * xx + math.sin(th) * yy) + phs)
    noise *= 8.0 / math.sqrt(n_waves / 2.0)
    return np.clip(img + noise, 0.0, 255.0)


def _fbm_canvas(cw: int, ch: int, rng: np.random.Generator, octaves: int = 6,
                persistence: float = 0.5, base_period: float = 64.0) -> np.ndarray:
    acc = torch.zeros((ch, cw), dtype=torch.float64)
    amp = 1.0
    period = base_period
    for _ in range(octaves):
        gw = int(math.ceil(cw / period)) + 4
        gh = int(math.ceil(ch / period)) + 4
        lat = torch.from_numpy(rng.uniform(-1.0, 1.0, size=(1, 1, gh, gw)))
        up = torch.nn.functional.interpolate(lat, scale_factor=period, mode="bicubic", align_corners=False)
        acc += amp * up[0, 0, :ch, :cw]
        amp *= persistence
        period /= 2.0
    a = acc.numpy()
    a = (a - a.mean()) / (a.std() + 1e-12)
    return np.clip(128.0 + 45.0 * a, 0.0, 255.0)


def _mover_textures(r: SeqRecipe, canvas: np.ndarray, rng: np.random.Generator) -> list:
    """Square patches cut from random places of the scene texture: the movers have the scene's
    statistics (so they do not dominate the corner scores) but move independently of the camera."""
    out = []
    s = r.mover_size
    ch, cw = canvas.shape
    for _ in range(r.n_movers):
        y0 = int(rng.integers(0, max(1, ch - s)))
        x0 = int(rng.integers(0, max(1, cw - s)))
        out.append(canvas[y0:y0 + s, x0:x0 + s].copy())
    return out


# ----------------------------------------------------------------------------------------------
# the sequence
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Sequence:
    recipe: SeqRecipe
    frames: object          # uint8 [n, H, W] (numpy array, or torch tensor on ``device``)
    A: np.ndarray           # world -> frame similarities, (n, 3, 3)

    @property
    def pair_transforms(self) -> np.ndarray:
        """S_j = A_{j+1} A_j^{-1}: frame-j pixel coords -> frame-(j+1) pixel coords, (n-1, 3, 3)."""
        return np.stack([self.A[j + 1] @ np.linalg.inv(self.A[j]) for j in range(len(self.A) - 1)])

    def pair_params_centred(self) -> np.ndarray:
        """Ground-truth (a, b, tx, ty) of each pair in centred coordinates x^ = x - (W-1)/2."""
        W, H = self.recipe.width, self.recipe.height
        cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
        C = np.array([[1, 0, -cx], [0, 1, -cy], [0, 0, 1.0]])
        Ci = np.linalg.inv(C)
        out = []
        for S in self.pair_transforms:
            Sc = C @ S @ Ci
            out.append([Sc[0, 0], Sc[1, 0], Sc[0, 2], Sc[1, 2]])
        return np.array(out)

    def mover_boxes(self):
        return self._movers


def make_sequence(name_or_recipe, n_frames: int | None = None, device: str | torch.device = "cpu",
                  as_numpy: bool = True) -> Sequence:
    """Render a seeded sequence. ``n_frames`` truncates the recipe's length (the camera chain is
    drawn for the full recipe first, so a prefix is identical to the full sequence's prefix)."""
    r = RECIPES[name_or_recipe] if isinstance(name_or_recipe, str) else name_or_recipe
    rng = np.random.default_rng(r.seed)
    A = _cameras(r, rng)
    n = r.n_frames if n_frames is None else min(n_frames, r.n_frames)
    W, H = r.width, r.height
    # world footprint of all frames (of the full recipe, so prefixes agree)
    corners = np.array([[0, 0, 1], [W - 1, 0, 1], [0, H - 1, 1], [W - 1, H - 1, 1]], dtype=np.float64).T
    pts = np.concatenate([(np.linalg.inv(A[j]) @ corners)[:2] for j in range(len(A))], axis=1)
    margin = 24
    ox = math.floor(pts[0].min()) - margin
    oy = math.floor(pts[1].min()) - margin
    cw = int(math.ceil(pts[0].max())) + margin - ox + 1
    ch = int(math.ceil(pts[1].max())) + margin - oy + 1
    if r.texture == "blobs":
        canvas = _blob_canvas(cw, ch, rng)
    else:
        canvas = _fbm_canvas(cw, ch, rng)
    movers = _mover_textures(r, canvas, rng)
    # movers are blended in with a raised-cosine border so their outline is not a hard step
    ramp = max(3, r.mover_size // 12)
    u = np.minimum(np.arange(r.mover_size) + 0.5, r.mover_size - np.arange(r.mover_size) - 0.5) / ramp
    w1 = 0.5 - 0.5 * np.cos(np.pi * np.clip(u, 0.0, 1.0))
    alpha_np = np.outer(w1, w1)
    # mover trajectories in frame coordinates: slow independent drift + wobble
    mpos = []
    for _ in range(r.n_movers):
        p0 = rng.uniform([0.15 * W, 0.15 * H], [0.85 * W - r.mover_size, 0.85 * H - r.mover_size])
        v = rng.normal(0.0, 1.5, size=2) * (r.mover_size / 40.0)
        wob = rng.uniform(2.0, 6.0) * (r.mover_size / 40.0)
        mpos.append((p0, v, wob, rng.uniform(0, 2 * math.pi)))

    dev = torch.device(device)
    dtype = torch.float32 if dev.type != "cpu" else torch.float64
    can = torch.from_numpy(canvas).to(device=dev, dtype=dtype)[None, None]
    alpha = torch.from_numpy(alpha_np).to(device=dev, dtype=dtype)
    ys, xs = torch.meshgrid(torch.arange(H, device=dev, dtype=dtype), torch.arange(W, device=dev, dtype=dtype),
                            indexing="ij")
    frames = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    for j in range(n):
        Ai = np.linalg.inv(A[j])
        wx = Ai[0, 0] * xs + Ai[0, 1] * ys + Ai[0, 2] - ox
        wy = Ai[1, 0] * xs + Ai[1, 1] * ys + Ai[1, 2] - oy
        grid = torch.stack([wx / (cw - 1) * 2 - 1, wy / (ch - 1) * 2 - 1], dim=-1)[None]
        v = torch.nn.functional.grid_sample(can, grid, mode="bicubic", padding_mode="border", align_corners=True)
        f = torch.clamp(torch.floor(v[0, 0] + 0.5), 0, 255)
        for (p0, vel, wob, ph), tex in zip(mpos, movers):
            s = r.mover_size
            px = p0[0] + vel[0] * j + wob * math.sin(0.21 * j + ph)
            py = p0[1] + vel[1] * j + wob * math.cos(0.17 * j + ph)
            # bounce inside the frame
            px = _reflect(px, 0.0, W - s - 1.0)
            py = _reflect(py, 0.0, H - s - 1.0)
            x0, y0 = int(round(px)), int(round(py))
            t = torch.from_numpy(tex).to(device=dev, dtype=f.dtype)
            blk = f[y0:y0 + s, x0:x0 + s]
            f[y0:y0 + s, x0:x0 + s] = torch.floor(alpha * t + (1 - alpha) * blk + 0.5)
        frames[j] = f.to(torch.uint8)
    out = frames.cpu().numpy() if (as_numpy and dev.type == "cpu") else frames
    seq = Sequence(r, out, A[:n])
    seq._movers = mpos
    return seq


def integer_translation_sequence(width: int, height: int, n_frames: int, max_step: int = 5,
                                 seed: int = 1709) -> Sequence:
    """Frames cut from one uint8 blob texture at integer offsets: frame j is the canvas window at
    offset o_j, o_0 = 0 and o_{j+1} - o_j drawn uniformly from [-max_step, max_step]^2. Every frame is
    an exact integer shift of the previous one (no resampling, no rounding), so the pair transform
    S_j is the translation by o_j - o_{j+1}, exactly."""
    rng = np.random.default_rng(seed)
    steps = rng.integers(-max_step, max_step + 1, size=(max(n_frames - 1, 0), 2))
    off = np.concatenate([np.zeros((1, 2), np.int64), np.cumsum(steps, axis=0)], axis=0)
    lo, hi = off.min(0), off.max(0)
    cw, ch = width + int(hi[0] - lo[0]), height + int(hi[1] - lo[1])
    canvas = np.clip(np.floor(_blob_canvas(cw, ch, rng) + 0.5), 0, 255).astype(np.uint8)
    frames = np.stack([canvas[int(o[1] - lo[1]):int(o[1] - lo[1]) + height, int(o[0] - lo[0]):int(o[0] - lo[0]) + width]
                       for o in off])
    A = np.stack([np.array([[1.0, 0.0, -float(o[0])], [0.0, 1.0, -float(o[1])], [0.0, 0.0, 1.0]]) for o in off])
    r = SeqRecipe("translate", width, height, n_frames, "blobs", "translate", seed=seed)
    seq = Sequence(r, np.ascontiguousarray(frames), A)
    seq._movers = []
    return seq


def _reflect(v: float, lo: float, hi: float) -> float:
    span = hi - lo
    if span <= 0:
        return lo
    t = (v - lo) % (2 * span)
    return lo + (t if t <= span else 2 * span - t)


# ----------------------------------------------------------------------------------------------
# small deterministic test images
# ----------------------------------------------------------------------------------------------

def random_image(w: int, h: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 256, size=(h, w), dtype=np.uint8)


def smooth_random_image(w: int, h: int, seed: int, sigma: float = 2.0) -> np.ndarray:
    """White noise blurred by a Gaussian (scipy), rescaled to [0, 255]: textured but smooth."""
    from scipy.ndimage import gaussian_filter
    a = np.random.default_rng(seed).normal(size=(h, w))
    a = gaussian_filter(a, sigma, mode="wrap")
    a = (a - a.min()) / (a.max() - a.min() + 1e-12)
    return np.clip(np.floor(a * 255.0 + 0.5), 0, 255).astype(np.uint8)


def random_points(n: int, w: int, h: int, margin: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(margin, w - 1 - margin, n), rng.uniform(margin, h - 1 - margin, n)], 1)
