"""Thin Python face of the serving runtime in libgsr (continuous batching of
render + L1 + backward + Adam requests against resident scenes). Every step
runs in the library; this module marshals arguments and writes checkpoints."""
from __future__ import annotations

import json
import os

import numpy as np

from . import gsr


def camera_struct(c) -> gsr.gsr_camera:
    return gsr.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.world_to_cam, c.znear, c.bg)


class Server:
    def __init__(self, budget_bytes: int, max_batch: int = 16, lanes: int = 2, config: gsr.gsr_config | None = None,
                 lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, device: int = 0,
                 capacity_render: bool = False):
        self.opts = gsr.make_server_opts(budget_bytes, max_batch, lanes, config, lr, beta1, beta2, eps,
                                         capacity_render)
        self.h = gsr.gsr_server_create(self.opts, device)
        self.meta = {}

    def close(self):
        if self.h is not None:
            gsr.gsr_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # scenes
    def add_scene(self, scene: gsr.gsr_scene) -> int:
        sid = gsr.gsr_server_add_scene(self.h, scene)
        self.meta[sid] = (int(scene.n), int(scene.sh_degree))
        return sid

    def remove_scene(self, sid: int):
        gsr.gsr_server_remove_scene(self.h, sid)
        self.meta.pop(sid, None)

    def block(self, sid: int, name: str) -> np.ndarray:
        n, d = self.meta[sid]
        out = np.empty(n * (11 + 3 * (d + 1) ** 2), np.float32)
        gsr.gsr_server_scene_io(self.h, sid, name, out, True)
        return out

    def step(self, sid: int) -> int:
        return gsr.gsr_server_scene_state(self.h, sid)[4]

    def save(self, sid: int, directory: str):
        """Checkpoint: the four flat blocks as .npy plus the step count."""
        os.makedirs(directory, exist_ok=True)
        n, d = self.meta[sid]
        for name in gsr.SCENE_BLOCKS:
            np.save(os.path.join(directory, f"{name}.npy"), self.block(sid, name))
        with open(os.path.join(directory, "scene.json"), "w") as f:
            json.dump({"n": n, "sh_degree": d, "step": self.step(sid)}, f)

    def load(self, directory: str) -> int:
        with open(os.path.join(directory, "scene.json")) as f:
            meta = json.load(f)
        sid = self.add_scene(gsr.gsr_scene(meta["n"], meta["sh_degree"], None, None, None, None, None))
        for name in gsr.SCENE_BLOCKS:
            arr = np.ascontiguousarray(np.load(os.path.join(directory, f"{name}.npy")), np.float32)
            gsr.gsr_server_scene_io(self.h, sid, name, arr, False)
        gsr.gsr_server_set_step(self.h, sid, meta["step"])
        return sid

    # requests
    @staticmethod
    def request(sid: int, camera, seed: int) -> gsr.gsr_request:
        return gsr.gsr_request(sid, camera_struct(camera), seed)

    def submit(self, req: gsr.gsr_request) -> int:
        return gsr.gsr_server_submit(self.h, req)

    def replay(self, reqs, arrival_s):
        return gsr.gsr_server_replay(self.h, reqs, arrival_s)

    def drain(self):
        gsr.gsr_server_drain(self.h)

    def results(self):
        return gsr.gsr_server_results(self.h)
