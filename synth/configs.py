"""The five synthetic workloads (sizes, seeds, render parameters)."""

from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class Config:
    name: str
    dims: tuple            # (nx, ny, nz)
    dtype: str             # "f32" | "f16"
    image: tuple           # (width, height)
    n_cams: int
    split: str             # "none" | "even" | "kd"
    parts: tuple = (1, 1, 1)
    n_bricks: int = 1
    n_blobs: int = 8
    s_range: tuple = (0.05, 0.2)
    a_range: tuple = (1.0, 1.0)
    log_sigma: bool = False
    noise: str = "white"   # "white" | "fbm"
    noise_amp: float = 0.02
    fbm_periods: tuple = ()
    step_voxels: float = 0.5
    ert: float = 0.99
    density: float = 20.0
    macrocell: int = 16
    seeds: dict = field(default_factory=dict)


CONFIGS = {
    "cfg1": Config("cfg1-single-64^3-f32", (64, 64, 64), "f32", (256, 256), 1, "none",
                   seeds=dict(volume=1001, tf=2001)),
    "cfg2": Config("cfg2-512^3-f32-2x2x2", (512, 512, 512), "f32", (1024, 1024), 1, "even",
                   parts=(2, 2, 2), n_bricks=8, seeds=dict(volume=1002, tf=2001)),
    "cfg3": Config("cfg3-1024x1024x768-f16-kd27-16cam", (1024, 1024, 768), "f16", (2048, 2048), 16, "kd",
                   n_bricks=27, n_blobs=64, s_range=(0.02, 0.12), a_range=(0.5, 1.0), noise="fbm",
                   noise_amp=0.15, fbm_periods=(128, 64, 32, 16, 8, 4),
                   seeds=dict(volume=1003, tf=2001, kd=3003)),
    "cfg4": Config("cfg4-256^3-f32-train-16cam", (256, 256, 256), "f32", (512, 512), 16, "none",
                   ert=1.0, seeds=dict(volume=1004, tf=2001, perturb=4004, fd=5004)),
    "cfg5": Config("cfg5-2048x1536x1280-f16-rank-share+K128", (2048, 1536, 1280), "f16", (3840, 2160), 1,
                   "none", n_blobs=256, s_range=(0.005, 0.2), a_range=(0.5, 1.0), log_sigma=True,
                   noise="fbm", noise_amp=0.15, fbm_periods=(512, 256, 128, 64, 32, 16, 8, 4),
                   seeds=dict(volume=1005, tf=2001, frames=6005)),
}


def get_config(key):
    return CONFIGS[key]
