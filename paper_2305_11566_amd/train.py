"""Training of the refinement network on coarse maps the matcher itself
produces (Sec. IV-A: Adam, beta1 = 0.99, beta2 = 0.999, lr = 5e-4; the loss
in the reading of Eqs. (9)-(11) used throughout: smooth-L1 + kl_weight * KL).

Every step runs on the GPU through libsv.so: census + WTA of the batch, the
training forward (with sampled reparameterisation noise), the loss and its
gradient, the hand-written backward, Adam on the FP32 master weights, and
the repack of the weights into the compute dtype.  Checkpoints hold the master
weights, both Adam moments and the step; the noise and the batch of a step
are functions of the step number, so a resumed run repeats the same steps.

    python -m paper_2305_11566_amd.train --steps 2000
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import ops
from .ops import Refiner, sv_census_pair, sv_cost_wta, sv_loss, sv_adam_step


def layer_shapes(c1, c2, c3, latent):
    """(out, in, k) per layer in the canonical order (for weight initialisation)."""
    return [(c1, 2, 3), (c2, c1, 3), (c3, c2, 3), (2 * latent, c3, 1), (c3, latent, 1),
            (c2, c3 + c2, 3), (c1, c2 + c1, 3), (c1, c1 + 2, 3), (1, c1 + 2, 3)]


class Trainer:
    def __init__(self, params: np.ndarray, C=(16, 32, 64), latent=64, factor=2, dtype="bf16",
                 win=(5, 5), D=16, lr=5e-4, beta1=0.99, beta2=0.999, eps=1e-8, kl_weight=1e-3,
                 eps_seed=9000, device="cuda"):
        self.C, self.L, self.f, self.win, self.D = tuple(C), latent, factor, tuple(win), D
        self.lr, self.b1, self.b2, self.adam_eps, self.klw = lr, beta1, beta2, eps, kl_weight
        self.eps_seed = eps_seed
        self.dev = torch.device(device)
        self.ref = Refiner(*C, latent, factor, dtype, device=device)
        self.w = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(self.dev)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.g = torch.empty_like(self.w)
        self.step = 0
        self._saved = {}
        self._loss_ws = torch.empty(ops.lib().sv_loss_workspace_bytes(), dtype=torch.uint8,
                                    device=self.dev)
        self.loss = torch.empty(3, dtype=torch.float32, device=self.dev)

    # -- pieces -------------------------------------------------------------------
    def coarse(self, left, right):
        nbits = self.win[0] * self.win[1] - 1
        cl, cr, low = sv_census_pair(left, right, self.f, *self.win)
        return sv_cost_wta(cl, cr, self.D, nbits), low

    def noise(self, B, H, W, step):
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(self.eps_seed + step)
        return torch.randn(self.ref.latent_shape(B, H, W), generator=gen, device=self.dev,
                           dtype=torch.float32)

    def train_step(self, left, right, gt):
        """One optimiser step on a batch (uint8 [B,H,W] x2, float32 gt [B,H,W])."""
        B, H, W = left.shape
        key = (B, H, W)
        if key not in self._saved:
            self._saved[key] = self.ref.saved_buffer(B, H, W)
        saved = self._saved[key]
        self.ref.pack(self.w)
        disp, low = self.coarse(left, right)
        eps = self.noise(B, H, W, self.step)
        out, ml = self.ref.forward(disp, low, H, W, eps=eps, saved=saved)
        _, dout = sv_loss(out, gt, ml, self.L, self.klw, loss_out=self.loss, workspace=self._loss_ws)
        self.ref.backward(saved, B, H, W, eps, dout, self.klw, grad=self.g)
        self.step += 1
        sv_adam_step(self.w, self.g, self.m, self.v, self.step, self.lr, self.b1, self.b2,
                     self.adam_eps)
        return self.loss

    @torch.no_grad()
    def evaluate(self, left, right, gt):
        """Mean end-point error (px) of the refined map and of the linear upscaling
        of the coarse map ("Mini+Linear"), against gt."""
        B, H, W = left.shape
        self.ref.pack(self.w)
        disp, low = self.coarse(left, right)
        out, _ = self.ref.forward(disp, low, H, W)
        lin = torch.nn.functional.interpolate(disp[:, None].float() * self.f, size=(H, W),
                                              mode="bilinear", align_corners=False)[:, 0]
        return (float((out - gt).abs().mean()), float((lin - gt).abs().mean()))

    # -- checkpoint / resume ----------------------------------------------------------
    def save(self, path):
        np.savez(path, w=self.w.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.int64(self.step))

    def load(self, path):
        z = np.load(path, allow_pickle=False)
        self.w.copy_(torch.from_numpy(z["w"]))
        self.m.copy_(torch.from_numpy(z["m"]))
        self.v.copy_(torch.from_numpy(z["v"]))
        self.step = int(z["step"])


class TableTrainer:
    """Training of the Table I network with the loss of Eqs. (9)-(11): census +
    WTA of the batch, the forward with the noise of Eq. (8), sv_tvae_loss,
    the hand-written backward, Adam on FP32 master weights, repack."""

    def __init__(self, params: np.ndarray, factor=2, dtype="bf16", win=(5, 5), D=16, lr=5e-4,
                 beta1=0.99, beta2=0.999, eps=1e-8, eps_seed=9000, device="cuda"):
        self.f, self.win, self.D = factor, tuple(win), D
        self.lr, self.b1, self.b2, self.adam_eps = lr, beta1, beta2, eps
        self.eps_seed = eps_seed
        self.dev = torch.device(device)
        self.net = ops.TableVAE(factor, dtype, device=device)
        self.w = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(self.dev)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.g = torch.empty_like(self.w)
        self.step = 0

    def coarse(self, left, right):
        nbits = self.win[0] * self.win[1] - 1
        cl, cr, low = sv_census_pair(left, right, self.f, *self.win)
        return sv_cost_wta(cl, cr, self.D, nbits), low

    def train_step(self, left, right, gt, noc, occ):
        """One optimiser step; gt float32 [B,H,W] px, noc / occ uint8 masks."""
        B, H, W = left.shape
        self.net.pack(self.w)
        disp, low = self.coarse(left, right)
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(self.eps_seed + self.step)
        eps = torch.randn(self.net.latent_shape(B, H, W), generator=gen, device=self.dev, dtype=torch.float32)
        out, ms = self.net.forward(disp, low, H, W, eps=eps)
        loss, dout, dms = ops.sv_tvae_loss(out, gt, noc, occ, ms)
        self.net.backward(disp, low, H, W, dout, eps=eps, dmu_sigma=dms, grad=self.g)
        self.step += 1
        sv_adam_step(self.w, self.g, self.m, self.v, self.step, self.lr, self.b1, self.b2, self.adam_eps)
        return loss


def make_pool(n, H, W, seed0, n_cells=6, dmin=4.0, dmax=24.0, device="cuda", masks=False):
    """Pairs, ground truth and (masks=True) the non-occluded / all-pixel masks as uint8."""
    from synth import gen_pair
    ps = [gen_pair(H, W, n_cells, dmin, dmax, seed=seed0 + i) for i in range(n)]
    t = lambda a, dt: torch.from_numpy(np.stack(a)).to(device=device, dtype=dt)
    base = (t([p.left for p in ps], torch.uint8), t([p.right for p in ps], torch.uint8),
            t([p.gt for p in ps], torch.float32))
    if not masks:
        return base
    return base + (t([p.noc for p in ps], torch.uint8), t([p.occ for p in ps], torch.uint8))


def batch_indices(step, batch, pool):
    """The pool entries used at a step (a function of the step only)."""
    rng = np.random.Generator(np.random.PCG64(123457 + step))
    return torch.from_numpy(rng.choice(pool, size=batch, replace=False))


def main():
    ap = argparse.ArgumentParser(description="train the refiner on synthetic 512x256 crops")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--dtype", default="bf16")
    ap.add_argument("--H", type=int, default=256)
    ap.add_argument("--W", type=int, default=512)
    ap.add_argument("--save", default="")
    ap.add_argument("--resume", default="")
    ap.add_argument("--log-every", type=int, default=100)
    args = ap.parse_args()
    from synth import he_init_params
    C, L = (16, 32, 64), 64
    params = he_init_params(layer_shapes(*C, L), seed=7005)
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])
    tr = Trainer(flat, C=C, latent=L, dtype=args.dtype)
    if args.resume:
        tr.load(args.resume)
    left, right, gt = make_pool(args.pool, args.H, args.W, seed0=5000)
    vl, vr, vg = make_pool(16, args.H, args.W, seed0=5500)
    print(json.dumps({"event": "start", "step": tr.step, "val_epe": tr.evaluate(vl, vr, vg)}), flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s0 = tr.step
    while tr.step < args.steps:
        idx = batch_indices(tr.step, args.batch, args.pool).to(left.device)
        loss = tr.train_step(left[idx], right[idx], gt[idx])
        if tr.step % args.log_every == 0:
            l = loss.cpu().numpy()
            el = time.perf_counter() - t0
            print(json.dumps({"event": "step", "step": tr.step, "loss": float(l[0]),
                              "data": float(l[1]), "kl": float(l[2]),
                              "steps_per_s": (tr.step - s0) / el}), flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    epe_ref, epe_lin = tr.evaluate(vl, vr, vg)
    print(json.dumps({"event": "done", "step": tr.step, "steps_per_s": (tr.step - s0) / max(el, 1e-9),
                      "val_epe_refined_px": epe_ref, "val_epe_linear_px": epe_lin}), flush=True)
    if args.save:
        tr.save(args.save)


if __name__ == "__main__":
    main()
