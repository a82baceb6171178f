"""Named synthetic workloads (scene, image shape, noise, table size).

Every workload is seeded (scene seed 1902; the multi-view workload uses
1902 + view for view v) and uses the same scene recipe; see synth.scene.

  tiny_64x64        64x64, 1 vertex per path, ground + 8 boxes, sigma 1,
                    table 2^14 slots.  Small enough for brute force.
  hd_1080p_x3       1920x1080, 3 vertices per path (6,220,800 slots),
                    ground + 8 boxes, sigma 1, table 2^22 slots,
                    16 frames of a camera orbiting 1 degree per frame,
                    exponential moving average with alpha_old = 0.2.
  uhd_4k_x4         3840x2160, 4 vertices per path (33,177,600 slots),
                    ground + 64 boxes + 16 spheres, sigma 1.5 with 1%
                    fireflies at 100x, table 2^25 slots.
  multiview_8       8 views (640x360, 1280x720, 3x 1920x1080, 2560x1440,
                    3840x2160, 800x600), 3 vertices per path each,
                    per-view tables of next_pow2(2 * W * H) slots.
  hd_1080p_x3_mlp   hd_1080p_x3 with the learned fallback for sparse cells.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .rng import M64, splitmix64
from .scene import camera_position, generate_view, make_scene

CONFIG_SEED = 1902


def frame_seed(config_seed: int, frame: int) -> int:
    """Per-frame 64-bit jitter seed handed to key construction."""
    return splitmix64((config_seed ^ frame) & M64)


@dataclass
class ViewSpec:
    width: int
    height: int
    verts_per_path: int
    log2_slots: int
    seed: int = CONFIG_SEED


@dataclass
class Workload:
    name: str
    views: list
    n_boxes: int = 8
    n_spheres: int = 0
    he_range: tuple = (0.3, 1.0)
    sigma: float = 1.0
    firefly_p: float = 0.0
    s: float = 0.01
    frames: int = 1
    orbit_deg: float = 1.0
    alpha_old: float = 0.2
    max_probe: int = 64
    frac_bits: int = 24
    extra: dict = field(default_factory=dict)

    @property
    def n_slots(self) -> int:
        return sum(v.width * v.height * v.verts_per_path for v in self.views)


def _next_pow2_log2(x: int) -> int:
    return max(4, (x - 1).bit_length())


WORKLOADS = {
    "tiny_64x64": Workload("tiny_64x64", [ViewSpec(64, 64, 1, 14)]),
    "hd_1080p_x3": Workload("hd_1080p_x3", [ViewSpec(1920, 1080, 3, 22)], frames=16),
    "uhd_4k_x4": Workload("uhd_4k_x4", [ViewSpec(3840, 2160, 4, 25)], n_boxes=64, n_spheres=16,
                          he_range=(0.2, 0.8), sigma=1.5, firefly_p=0.01),
    "multiview_8": Workload("multiview_8", [
        ViewSpec(w, h, 3, _next_pow2_log2(2 * w * h), CONFIG_SEED + i)
        for i, (w, h) in enumerate([(640, 360), (1280, 720), (1920, 1080), (1920, 1080), (1920, 1080),
                                    (2560, 1440), (3840, 2160), (800, 600)])]),
    "hd_1080p_x3_mlp": Workload("hd_1080p_x3_mlp", [ViewSpec(1920, 1080, 3, 22)], frames=16,
                                extra={"mlp": True}),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]


def generate(wl: Workload, view: int = 0, frame: int = 0, device="cpu", width=None, height=None):
    """Vertex streams of one view and frame, plus its filter parameters.

    width/height override the view's image size (for scaled-down tests);
    everything else, including the seeds, stays as in the workload.
    """
    v = wl.views[view]
    scene = make_scene(v.seed, wl.n_boxes, wl.n_spheres, wl.he_range)
    eye = camera_position(frame, wl.orbit_deg)
    out = generate_view(scene, width or v.width, height or v.height, v.verts_per_path, eye,
                        v.seed, frame, wl.sigma, wl.firefly_p, device=device)
    out["seed"] = frame_seed(v.seed, frame)
    out["s"] = wl.s
    out["log2_slots"] = v.log2_slots
    out["max_probe"] = wl.max_probe
    out["frac_bits"] = wl.frac_bits
    return out
