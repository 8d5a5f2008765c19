"""Training of the learned flip scorer on frames the decoder generates.

Every step: the channel kernel draws a batch of frames at Eb/N0 uniform in
[lo, hi] dB (per-frame noise level), the learned decoder runs on them with
the current parameters and emits one record per scored proposal (features
and the label z xor c), the scorer kernels compute the gradient of the
weighted binary cross-entropy over the records (fixed-order reduction), and
an Adam step updates the float32 parameters.  All of it runs in the
library's HIP kernels; this module only sequences the calls and keeps the
device buffers.  Checkpoints hold the parameters, both Adam moments, the step
count and the generator counters, as a numpy .npz file.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np

from . import fwbf, synth

H = 32


def init_params(rounds: int, alpha: float = 0.2, seed: int = 7) -> np.ndarray:
    """He-initialised weights; alpha_t = alpha, beta_t = 1 (the plain metric)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.normal(0, np.sqrt(2.0 / 4), (H, 4))
    b1 = np.zeros(H)
    W2 = rng.normal(0, np.sqrt(2.0 / H), (H, H))
    b2 = np.zeros(H)
    W3 = rng.normal(0, np.sqrt(1.0 / H), H)
    b3 = np.zeros(1)
    al = np.full(rounds, alpha)
    be = np.ones(rounds)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, b3, al, be]).astype(np.float32)


@dataclasses.dataclass
class TrainConfig:
    rounds: int = 16
    groups: int = 32
    topk: int = 1
    batch: int = 1 << 13
    steps: int = 200
    lr: float = 2e-3
    pos_weight: float = 1.0
    ebn0_lo: float = 3.0
    ebn0_hi: float = 5.0
    seed: int = 7
    pool_size: int = 1024
    plain_groups: int = 8
    max_iter: int = 100
    int16: bool = False    # int16 frames (scale 256) instead of int8 (scale 16)


class Trainer:
    def __init__(self, code: fwbf.Code, cfg: TrainConfig, device="cuda"):
        import torch
        self.torch = torch
        self.code, self.cfg, self.dev = code, cfg, device
        # the device comes up through torch before the library's first call
        self.params = torch.from_numpy(init_params(cfg.rounds, seed=cfg.seed)).to(device)
        self.scale = 256.0 if cfg.int16 else 16.0
        self.lp = fwbf.LearnedParams(cfg.rounds, cfg.groups, cfg.topk, self.scale)
        self.P = fwbf.scorer_size(cfg.rounds)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros(self.P + 2, dtype=torch.float32, device=device)
        self.work = torch.empty(1024 * (self.P + 2), dtype=torch.float32, device=device)
        self.step_count = 0
        pool = code.encode(seed=cfg.seed * 1000 + 1, first=0, count=cfg.pool_size)
        self.pool = torch.from_numpy(pool.view(np.int32)).to(device)
        self.plain = fwbf.DecodeParams(dtype=fwbf.I16 if cfg.int16 else fwbf.I8, groups=cfg.plain_groups,
                                       max_iter=cfg.max_iter, alpha_num=1, alpha_den=5)
        B = cfg.batch
        self.y = torch.empty((B, code.N), dtype=torch.int16 if cfg.int16 else torch.int8, device=device)
        self.sig = torch.empty(B, dtype=torch.float32, device=device)
        self.rec = fwbf.record_buffer(B, cfg.rounds, cfg.groups, cfg.topk, device)
        self.z = torch.empty((B, (code.N + 31) // 32), dtype=torch.int32, device=device)
        self.it = torch.empty(B, dtype=torch.int32, device=device)
        self.ok = torch.empty(B, dtype=torch.uint8, device=device)
        self.lok = torch.empty(B, dtype=torch.uint8, device=device)
        self.history = []

    def _frames(self, f0: int):
        cfg = self.cfg
        eb = synth.uniform_frames(self.code.N, cfg.batch, cfg.seed + f0, cfg.ebn0_lo, cfg.ebn0_hi)
        sig = synth.sigma_for(eb, self.code.rate).astype(np.float32)
        self.sig.copy_(self.torch.from_numpy(sig))
        fwbf.channel_into(self.code.N, self.y, f0, self.pool, seed=cfg.seed * 7919, stream_id=9,
                          sigma=0.0, sigma_per_frame=self.sig, scale=self.scale)

    def step(self):
        cfg = self.cfg
        f0 = self.step_count * cfg.batch
        self._frames(f0)
        fwbf.decode_learned_into(self.code, self.y, self.plain, self.lp, self.params, self.z,
                                 self.it, self.ok, self.lok, self.rec, self.pool, f0)
        tiles = cfg.batch * cfg.rounds * fwbf.record_slots(cfg.groups, cfg.topk) // 32
        fwbf.scorer_grad(self.rec, tiles, self.lp, self.params, cfg.pos_weight,
                         out=self.grad, workspace=self.work)
        self.step_count += 1
        fwbf.adam(self.params, self.grad, self.m, self.v, self.step_count, cfg.lr)

    def train(self, steps=None, log_every=0):
        for s in range(steps or self.cfg.steps):
            self.step()
            if log_every and (s % log_every == 0):
                g = self.grad.cpu().numpy()
                self.history.append((self.step_count, float(g[self.P]), int(g[self.P + 1]),
                                     float(self.lok.float().mean().item())))
        return self

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), step=self.step_count,
                 config=np.array(list(dataclasses.asdict(self.cfg).items()), dtype=object).astype(str))

    def load(self, path):
        d = np.load(path, allow_pickle=False)
        self.params.copy_(self.torch.from_numpy(d["params"]))
        self.m.copy_(self.torch.from_numpy(d["m"]))
        self.v.copy_(self.torch.from_numpy(d["v"]))
        self.step_count = int(d["step"])


# the codes a scorer is trained for: (mb, nb, Z, seed) and their defaults
CODES = {
    "n1008": dict(code=(3, 6, 168, 2), int16=False, groups=32, plain_groups=8, batch=1 << 13,
                  ebn0_lo=3.0, ebn0_hi=5.0),
    "n32400": dict(code=(3, 30, 1080, 5), int16=True, groups=512, plain_groups=16, batch=1 << 10,
                   ebn0_lo=5.0, ebn0_hi=7.0),
}


def main(argv=None):
    """Train the scorer of one code on the GPU and write a checkpoint:
    python -m paper_1206_3362_amd.learned --code n1008 --steps 512 --out x.npz"""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--code", choices=sorted(CODES), default="n1008",
                    help="n1008: (3,6) Z=168 int8; n32400: (3,30) Z=1080 int16")
    ap.add_argument("--steps", type=int, default=512, help="steps of --batch frames (512 x 8192 = 2^22)")
    ap.add_argument("--batch", type=int, default=0, help="frames per step (0: the code's default)")
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--rounds", type=int, default=16)
    ap.add_argument("--groups", type=int, default=0, help="blocks of the learned pass (0: the code's default)")
    ap.add_argument("--topk", type=int, default=1)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch
    torch.zeros(1, device="cuda")  # bring the device up before the library loads
    d = CODES[a.code]
    code = fwbf.Code.from_seed(*d["code"])
    cfg = TrainConfig(rounds=a.rounds, groups=a.groups or d["groups"], topk=a.topk, batch=a.batch or d["batch"],
                      steps=a.steps, lr=a.lr, seed=a.seed, int16=d["int16"], plain_groups=d["plain_groups"],
                      ebn0_lo=d["ebn0_lo"], ebn0_hi=d["ebn0_hi"])
    tr = Trainer(code, cfg).train(log_every=max(1, a.steps // 16))
    tr.torch.cuda.synchronize()
    for step, loss, records, lpass in tr.history:
        print(f"step {step}: loss {loss:.4f} records {records} learned-pass decoded {lpass:.3f}", flush=True)
    tr.save(a.out)


if __name__ == "__main__":
    main()
