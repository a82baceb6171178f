"""Procedural scenes and path-vertex streams (phase one of the method).

The method filters a set of path vertices produced by a renderer (the two
phase pipeline at the start of the Algorithm section).  No renderer or scene
from the paper is available, so this module makes one: a ground plane y = 0
plus seeded axis-aligned boxes (and spheres for the 4K scene), a pinhole
camera, one path per pixel with cosine-sampled bounces, and per-vertex
"contributions" (Eq. (9)'s L_i * f_i * cos) equal to
albedo * max(0, n . l) times a mean-one noise multiplier.  The noise-free
value albedo * max(0, n . l) is returned as the truth, and each vertex's path
throughput (the product of the albedos before it on its path) as tr, tg, tb,
so that sum over a pixel's vertices of throughput times contribution forms
its image.

Vertex streams are bounce-major structure-of-arrays: slot b * W * H + pixel
holds bounce b of the path through that pixel, pixels in row-major order.
Rays that leave the scene mark their vertex and all later ones invalid.

Nothing here is part of the filter; only inputs are made.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from .rng import HostRng, derive_key, rand_normal, rand_uniform

LIGHT_DIR = (0.4, 1.0, -0.6)
GROUND_ALBEDO = 0.5
EPS_T = 1e-4          # minimum ray parameter accepted as a hit
ORIGIN_OFFSET = 1e-4  # bounce origins are pushed off the surface by this


@dataclass
class Scene:
    box_lo: list = field(default_factory=list)      # [B][3]
    box_hi: list = field(default_factory=list)      # [B][3]
    box_albedo: list = field(default_factory=list)  # [B][3]
    sph_c: list = field(default_factory=list)       # [S][3]
    sph_r: list = field(default_factory=list)       # [S]
    sph_albedo: list = field(default_factory=list)  # [S][3]


def make_scene(seed: int, n_boxes: int, n_spheres: int = 0,
               he_range=(0.3, 1.0)) -> Scene:
    """Seeded boxes with centres in [-4, 4]^3, resting at or above y = 0."""
    rng = HostRng(derive_key(seed, 0x5CE4E))
    sc = Scene()
    lo_he, hi_he = he_range
    for _ in range(n_boxes):
        he = [lo_he + (hi_he - lo_he) * rng.uniform() for _ in range(3)]
        cx = -4.0 + 8.0 * rng.uniform()
        cz = -4.0 + 8.0 * rng.uniform()
        cy = he[1] + (4.0 - he[1]) * rng.uniform()
        c = [cx, cy, cz]
        sc.box_lo.append([c[i] - he[i] for i in range(3)])
        sc.box_hi.append([c[i] + he[i] for i in range(3)])
        sc.box_albedo.append([0.1 + 0.8 * rng.uniform() for _ in range(3)])
    for _ in range(n_spheres):
        r = 0.2 + 0.4 * rng.uniform()
        c = [-4.0 + 8.0 * rng.uniform(), r + (4.0 - r) * rng.uniform(), -4.0 + 8.0 * rng.uniform()]
        sc.sph_c.append(c)
        sc.sph_r.append(r)
        sc.sph_albedo.append([0.1 + 0.8 * rng.uniform() for _ in range(3)])
    return sc


def camera_position(frame: int, orbit_deg: float = 1.0, base=(0.0, 2.0, -6.0)):
    """Eye position rotated about +y by frame * orbit_deg degrees."""
    th = math.radians(frame * orbit_deg)
    x, y, z = base
    return (x * math.cos(th) + z * math.sin(th), y, -x * math.sin(th) + z * math.cos(th))


def _normalize(v):
    n = math.sqrt(sum(c * c for c in v))
    return tuple(c / n for c in v)


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _trace(o, d, scene: Scene, device):
    """Closest hit of rays (o, d) [N,3] float32: returns t, pos, n, albedo, hit."""
    N = o.shape[0]
    inf = torch.tensor(float("inf"), device=device)
    t_best = torch.full((N,), float("inf"), device=device)
    pos = torch.zeros((N, 3), device=device)
    nrm = torch.zeros((N, 3), device=device)
    alb = torch.zeros((N, 3), device=device)

    # ground plane y = 0, seen from above
    dy = d[:, 1]
    tg = torch.where(dy < 0, -o[:, 1] / torch.where(dy < 0, dy, -torch.ones_like(dy)), inf)
    tg = torch.where((o[:, 1] > 0) & (tg > EPS_T), tg, inf)
    m = tg < t_best
    if m.any():
        t_best = torch.where(m, tg, t_best)
        p = o + tg[:, None] * d
        p[:, 1] = 0.0                     # exactly on the plane
        pos = torch.where(m[:, None], p, pos)
        nrm = torch.where(m[:, None], torch.tensor([0.0, 1.0, 0.0], device=device), nrm)
        alb = torch.where(m[:, None], torch.full((3,), GROUND_ALBEDO, device=device), alb)

    # axis-aligned boxes (slab test); hits from outside only
    dsafe = torch.where(d.abs() < 1e-20, torch.full_like(d, 1e-20), d)
    inv = 1.0 / dsafe
    for lo_l, hi_l, al in zip(scene.box_lo, scene.box_hi, scene.box_albedo):
        lo = torch.tensor(lo_l, device=device)
        hi = torch.tensor(hi_l, device=device)
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
        tmin = torch.minimum(t1, t2)
        tmax = torch.maximum(t1, t2)
        tnear, axis = tmin.max(dim=1)
        tfar = tmax.min(dim=1).values
        hit = (tnear <= tfar) & (tnear > EPS_T)
        m = hit & (tnear < t_best)
        if not m.any():
            continue
        t_best = torch.where(m, tnear, t_best)
        p = o + tnear[:, None] * d
        onehot = torch.nn.functional.one_hot(axis, 3).to(torch.bool)
        dax = torch.gather(d, 1, axis[:, None])[:, 0]
        face = torch.where(dax > 0, lo[axis], hi[axis])  # entered through lo face when moving +
        p = torch.where(onehot, face[:, None], p)          # exactly on the face
        sgn = torch.where(dax > 0, -1.0, 1.0)
        nn_ = onehot.to(torch.float32) * sgn[:, None]
        pos = torch.where(m[:, None], p, pos)
        nrm = torch.where(m[:, None], nn_, nrm)
        alb = torch.where(m[:, None], torch.tensor(al, device=device), alb)

    for c_l, r, al in zip(scene.sph_c, scene.sph_r, scene.sph_albedo):
        c = torch.tensor(c_l, device=device)
        oc = o - c
        b = (oc * d).sum(1)
        cc = (oc * oc).sum(1) - r * r
        disc = b * b - cc
        ts = -b - torch.sqrt(torch.clamp(disc, min=0.0))
        m = (disc > 0) & (ts > EPS_T) & (ts < t_best)
        if not m.any():
            continue
        t_best = torch.where(m, ts, t_best)
        p = o + ts[:, None] * d
        n_ = (p - c) / r
        n_ = n_ / n_.norm(dim=1, keepdim=True)
        pos = torch.where(m[:, None], p, pos)
        nrm = torch.where(m[:, None], n_, nrm)
        alb = torch.where(m[:, None], torch.tensor(al, device=device), alb)

    hit = torch.isfinite(t_best)
    return pos, nrm, alb, hit


def _cosine_direction(n, u1, u2):
    """Cosine-weighted direction about unit normals n [N,3].

    Tangent frame from Duff et al., "Building an Orthonormal Basis,
    Revisited", JCGT 6(1), 2017.
    """
    sign = torch.where(n[:, 2] >= 0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = torch.stack([1.0 + sign * n[:, 0] * n[:, 0] * a, sign * b, -sign * n[:, 0]], 1)
    bt = torch.stack([b, sign + n[:, 1] * n[:, 1] * a, -n[:, 1]], 1)
    r = torch.sqrt(u1)
    phi = 2.0 * math.pi * u2
    z = torch.sqrt(torch.clamp(1.0 - u1, min=0.0))
    d = (r * torch.cos(phi))[:, None] * t + (r * torch.sin(phi))[:, None] * bt + z[:, None] * n
    return d / d.norm(dim=1, keepdim=True)


def generate_view(scene: Scene, width: int, height: int, verts_per_path: int,
                  eye, seed: int, frame: int, sigma: float = 1.0,
                  firefly_p: float = 0.0, fov_deg: float = 60.0,
                  device="cpu") -> dict:
    """One frame of bounce-major SoA vertex streams for one view."""
    device = torch.device(device)
    P = width * height
    N = P * verts_per_path
    pix = torch.arange(P, device=device, dtype=torch.int64)
    px = (pix % width).to(torch.float32)
    py = (pix // width).to(torch.float32)
    fkey = derive_key(seed, frame)
    jx = rand_uniform(derive_key(fkey, 11), pix)
    jy = rand_uniform(derive_key(fkey, 12), pix)

    eye_t = torch.tensor(eye, dtype=torch.float32, device=device)
    fwd = _normalize(tuple(-c for c in eye))              # looking at the origin
    right = _normalize(_cross((0.0, 1.0, 0.0), fwd))
    up = _cross(fwd, right)
    tan_half = math.tan(math.radians(fov_deg) * 0.5)
    aspect = width / height
    sx = (2.0 * (px + jx) / width - 1.0) * aspect * tan_half
    sy = (1.0 - 2.0 * (py + jy) / height) * tan_half
    d = (torch.tensor(fwd, device=device)[None, :]
         + sx[:, None] * torch.tensor(right, device=device)[None, :]
         + sy[:, None] * torch.tensor(up, device=device)[None, :])
    d = d / d.norm(dim=1, keepdim=True)
    o = eye_t.expand(P, 3).contiguous()

    light = torch.tensor(_normalize(LIGHT_DIR), dtype=torch.float32, device=device)
    pos_all = torch.zeros((N, 3), device=device)
    nrm_all = torch.zeros((N, 3), device=device)
    rgb_all = torch.zeros((N, 3), device=device)
    truth_all = torch.zeros((N, 3), device=device)
    valid_all = torch.zeros((N,), dtype=torch.uint8, device=device)
    tput_all = torch.zeros((N, 3), device=device)
    # path throughput of each vertex: the product of the albedos of the
    # earlier vertices of its path (the cosine of a cosine-sampled bounce
    # cancels its density, and the lambertian 1/pi cancels the pi of the
    # density's normalisation); 1 for the first hit of the camera ray
    tput = torch.ones((P, 3), device=device)

    alive = torch.ones((P,), dtype=torch.bool, device=device)
    for b in range(verts_per_path):
        pos, nrm, alb, hit = _trace(o, d, scene, device)
        ok = alive & hit
        sl = slice(b * P, (b + 1) * P)
        cosl = torch.clamp((nrm * light).sum(1), min=0.0)
        truth = alb * cosl[:, None]
        vid = pix + b * P
        z = rand_normal(derive_key(fkey, 21), vid)
        mult = torch.exp(sigma * z - 0.5 * sigma * sigma)
        if firefly_p > 0.0:
            u = rand_uniform(derive_key(fkey, 22), vid)
            mult = mult * torch.where(u < firefly_p, 100.0, 1.0) / (1.0 + 99.0 * firefly_p)
        okf = ok[:, None]
        pos_all[sl] = torch.where(okf, pos, 0.0)
        nrm_all[sl] = torch.where(okf, nrm, 0.0)
        truth_all[sl] = torch.where(okf, truth, 0.0)
        rgb_all[sl] = torch.where(okf, truth * mult[:, None], 0.0)
        valid_all[sl] = ok.to(torch.uint8)
        tput_all[sl] = torch.where(okf, tput, 0.0)
        tput = tput * alb
        alive = ok
        if b + 1 < verts_per_path:
            u1 = rand_uniform(derive_key(fkey, 31 + 2 * b), pix)
            u2 = rand_uniform(derive_key(fkey, 32 + 2 * b), pix)
            d = _cosine_direction(torch.where(ok[:, None], nrm, torch.tensor([0.0, 1.0, 0.0], device=device)), u1, u2)
            o = pos + ORIGIN_OFFSET * nrm

    return {
        "px": pos_all[:, 0].contiguous(), "py": pos_all[:, 1].contiguous(), "pz": pos_all[:, 2].contiguous(),
        "nx": nrm_all[:, 0].contiguous(), "ny": nrm_all[:, 1].contiguous(), "nz": nrm_all[:, 2].contiguous(),
        "r": rgb_all[:, 0].contiguous(), "g": rgb_all[:, 1].contiguous(), "b": rgb_all[:, 2].contiguous(),
        "valid": valid_all,
        "truth": truth_all,
        "tr": tput_all[:, 0].contiguous(), "tg": tput_all[:, 1].contiguous(), "tb": tput_all[:, 2].contiguous(),
        "cam": tuple(float(torch.tensor(c, dtype=torch.float32)) for c in eye),
        "width": width, "height": height, "verts_per_path": verts_per_path,
    }
