"""Learned initial guess: training data from the library's own solves, GPU training,
and solves that start from the network's corrections.

Every numerical step runs in the library (include/bsm.h, include/bsm_guess.h);
this module only sequences the calls.  The networks predict corrections to the
method's plain starts, block by block from pair descriptors:
    Z0 = I / rho + scale_Z * netZ(x_ij)     on P_Z   (Hotelling, guarded)
    L0 = c mask_L(Z) + scale_L * netL(x_ij) on P_L   (LNV, guarded)
Training targets are the differences between converged and plain starts of
solves the library ran itself.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import bsm as B


def init_params(out_dim: int, seed: int, width: int = B.MLP_WIDTH) -> np.ndarray:
    """Glorot-uniform hidden layers, zero biases and a zero output layer (so the
    untrained network predicts no correction: the plain starts)."""
    rng = np.random.default_rng(seed)
    D, H = B.DESC_DIM, width
    l1, l2 = np.sqrt(6.0 / (D + H)), np.sqrt(6.0 / (2 * H))
    parts = [rng.uniform(-l1, l1, D * H), np.zeros(H), rng.uniform(-l2, l2, H * H), np.zeros(H),
             np.zeros(H * out_dim), np.zeros(out_dim)]
    return np.concatenate(parts).astype(np.float32)


class Frame:
    """One system on the GPU: patterns P_S (= P_H), P_Z, P_L and the matrices S, H, Z, L."""

    def __init__(self, ctx: B.Context, system):
        self.ctx, self.sys = ctx, system
        cut, b = system.cutoffs, system.b
        pos = torch.tensor(system.positions, dtype=torch.float64, device=ctx.device)
        self.PS = B.Pattern(ctx, pos, system.box, cut["S"], b)
        self.PZ = B.Pattern(ctx, pos, system.box, cut["Z"], b)
        self.PL = B.Pattern(ctx, pos, system.box, cut["L"], b)
        self.S, self.H = B.Matrix(self.PS), B.Matrix(self.PS)
        B.fill_blocks(self.S, system.S.rows, system.S.cols, system.S.blocks)
        B.fill_blocks(self.H, system.H.rows, system.H.cols, system.H.blocks)
        self.Z, self.L = B.Matrix(self.PZ), B.Matrix(self.PL)
        self.lnv: Optional[B.LNV] = None

    def _lnv(self, tol_E):
        if self.lnv is None:
            self.lnv = B.LNV(self.S, self.H, self.Z, self.L, self.sys.n_electrons, tol_E=tol_E, init_from_z=False)
        self.lnv.tol_E = float(tol_E)
        return self.lnv

    def iterate(self, max_iter: int, tol_E: float):
        """LNV steps from the current start until |dE| < tol_E; returns (steps, last result)."""
        res = None
        for it in range(1, max_iter + 1):
            res = self.lnv.step(raise_on_error=True)
            if res.converged:
                return it, res
        raise RuntimeError(f"LNV did not converge in {max_iter} steps")

    def run_schedule(self, schedule):
        """LNV from the current start through a precision schedule (bsm.LNV.solve stages);
        returns (steps, result dict)."""
        r = self.lnv.solve(schedule)
        if r["status"] != 0 or not r["converged"]:
            raise RuntimeError(f"LNV schedule ended with status {r['status']}, converged {r['converged']}")
        return sum(r["iterations"]), r

    def release_state(self):
        """Free the LNV solver state (its matrices return to the allocator): for systems whose
        state and Hotelling's temporaries do not fit on the device together."""
        self.close()
        torch.cuda.empty_cache()

    def solve_plain(self, tol_E: float = 1e-8, max_iter: int = 300, fresh_state: bool = False,
                    schedule=None) -> dict:
        """Hotelling from I / rho, LNV from c mask_L(Z); keeps the plain starts for targets.
        fresh_state: release the previous solve's LNV state before Hotelling runs.
        schedule: LNV precision stages (bsm.LNV.solve) instead of FP64 steps to tol_E."""
        if fresh_state:
            self.release_state()
        t = time.perf_counter()
        hr = B.hotelling_inverse(self.S, self.Z, init_given=B.INIT_PLAIN)
        lnv = self._lnv(tol_E)
        lnv.reset(init_from_z=True)
        self.L_plain = B.Matrix(self.PL, self.L.blocks.clone())
        if schedule is None:
            steps, res = self.iterate(max_iter, tol_E)
            E, N = res.E, res.N
        else:
            steps, r = self.run_schedule(schedule)
            E, N = r["E"], r["N"]
        torch.cuda.synchronize()
        self.alpha = hr.alpha
        return dict(hotelling=hr.iterations, lnv=steps, E=E, N=N, seconds=time.perf_counter() - t)

    def solve_guess(self, netZ: "GuessNet", netL: "GuessNet", tol_E: float = 1e-8, max_iter: int = 300,
                    precision: int = B.BF16, n_tol: float = 0.01, fresh_state: bool = False,
                    schedule=None) -> dict:
        """Hotelling and LNV from the networks' corrected starts (each guarded by the plain one).
        fresh_state, schedule: as in solve_plain."""
        if fresh_state:
            self.release_state()
        t = time.perf_counter()
        XZ = B.pair_descriptors(self.PS, self.PZ)
        netZ.net.predict_blocks(XZ, self.Z, scale=netZ.scale, beta=0.0, precision=precision)
        B.symmetrize(self.Z)
        hr = B.hotelling_inverse(self.S, self.Z, init_given=B.INIT_GUARDED)
        XL = B.pair_descriptors(self.PS, self.PL)
        dL = B.Matrix(self.PL)
        netL.net.predict_blocks(XL, dL, scale=netL.scale, beta=0.0, precision=precision)
        B.symmetrize(dL)
        lnv = self._lnv(tol_E)
        g = lnv.reset_guess(dL, n_tol=n_tol)
        if schedule is None:
            steps, res = self.iterate(max_iter, tol_E)
            E, N = res.E, res.N
        else:
            steps, r = self.run_schedule(schedule)
            E, N = r["E"], r["N"]
        torch.cuda.synchronize()
        return dict(hotelling=hr.iterations, hotelling_start=hr.start, lnv=steps, accepted=g["accepted"],
                    E_start_plain=g["E_plain"], E_start_guess=g["E_guess"], E=E, N=N,
                    seconds=time.perf_counter() - t)

    def samples(self, scale_Z: float, scale_L: float):
        """Descriptors and targets of the last plain solve: (XZ, TZ, XL, TL)."""
        Zb = B.Matrix(self.PZ)
        B.set_identity(Zb, self.alpha)
        XZ = B.pair_descriptors(self.PS, self.PZ)
        TZ = B.mlp_targets(self.Z, Zb, scale_Z)
        XL = B.pair_descriptors(self.PS, self.PL)
        TL = B.mlp_targets(self.L, self.L_plain, scale_L)
        return XZ, TZ, XL, TL

    def correction_rms(self):
        """RMS element of Z* - I / rho and of L* - c mask_L(Z) after a plain solve."""
        Zb = B.Matrix(self.PZ)
        B.set_identity(Zb, self.alpha)
        B.axpby(1.0, self.Z, -1.0, Zb)
        dL = B.Matrix(self.PL, self.L.blocks.clone())
        B.axpby(-1.0, self.L_plain, 1.0, dL)
        nz, nl = Zb.blocks.numel(), dL.blocks.numel()
        return float(np.sqrt(B.dot(Zb, Zb) / nz)), float(np.sqrt(B.dot(dL, dL) / nl))

    def close(self):
        if self.lnv is not None:
            self.lnv.close()
            self.lnv = None


@dataclasses.dataclass
class GuessNet:
    net: B.MLP
    scale: float


def train_guess(ctx: B.Context, frames, epochs: int = 40, batch: int = 4096, lr: float = 1e-3,
                seed: int = 0, log=None, sample_frac: float = 1.0, close_frames: bool = False):
    """Train the Z and L networks on plain solves of `frames` (solved here, one after the
    other).  `frames` holds Frames or zero-argument callables that build one; with
    close_frames each frame is released once its samples are taken, so only one solver
    state is alive at a time.  sample_frac < 1 keeps that seeded fraction of each frame's
    pair samples.  Returns (netZ, netL, info) with per-epoch losses and the solves'
    iteration counts."""
    solves, data = [], []
    scale_Z = scale_L = None
    b2 = None
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)

    def keep(X, T):
        if sample_frac >= 1.0:
            return X, T
        n = X.shape[0]
        idx = torch.randperm(n, generator=gen)[:max(1, int(round(sample_frac * n)))].to(X.device)
        return X.index_select(0, idx), T.index_select(0, idx)

    for k, fr in enumerate(frames):
        f = fr() if callable(fr) else fr
        solves.append(f.solve_plain())
        if scale_Z is None:
            rz, rl = f.correction_rms()
            scale_Z, scale_L = max(rz, 1e-30), max(rl, 1e-30)
        XZ, TZ, XL, TL = f.samples(scale_Z, scale_L)
        data.append(keep(XZ, TZ) + keep(XL, TL))
        b2 = f.sys.b ** 2
        if log:
            r = solves[-1]
            log(f"[guess] training frame {k}: {f.sys.natoms} atoms, {r['hotelling']} + {r['lnv']} steps in "
                f"{r['seconds']:.2f} s, {data[-1][0].shape[0]} Z and {data[-1][2].shape[0]} L samples kept")
        if close_frames:
            f.close()
            del f
            torch.cuda.empty_cache()
    XZ = torch.cat([d[0] for d in data])
    TZ = torch.cat([d[1] for d in data])
    XL = torch.cat([d[2] for d in data])
    TL = torch.cat([d[3] for d in data])
    del data
    out = []
    for name, X, T, scale in (("Z", XZ, TZ, scale_Z), ("L", XL, TL, scale_L)):
        net = B.MLP(ctx, b2, init_params(b2, seed + (name == "L")))
        perm = torch.randperm(X.shape[0], generator=gen).to(torch.int32).to(ctx.device)
        t = time.perf_counter()
        losses = net.train(X, T, epochs=epochs, batch=batch, lr=lr, perm=perm)
        torch.cuda.synchronize()
        if log:
            log(f"[guess] net{name}: {X.shape[0]} samples, loss {losses[0]:.4g} -> {losses[-1]:.4g} "
                f"in {time.perf_counter() - t:.1f} s")
        out.append((GuessNet(net, scale), losses, X.shape[0]))
    info = dict(solves=solves, scale_Z=scale_Z, scale_L=scale_L, losses_Z=out[0][1], losses_L=out[1][1],
                samples_Z=out[0][2], samples_L=out[1][2])
    return out[0][0], out[1][0], info
