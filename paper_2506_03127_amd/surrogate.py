"""Learned surrogate of rho(t) over a box of bath and system parameters.

A network maps (w0, gamma, lambda, alpha, eps, t) -- the Brownian-oscillator
peak's frequency, width and reorganisation energy, the Ohmic coupling, the
bias of H_S = (eps/2) sigma_z + (Delta/2) sigma_x, and the time -- to the four
real components of rho(t) (rho_00, Re rho_01, Im rho_01, rho_11).  It is
trained on trajectories of the batched propagation (one instance per
parameter point) with the library's network kernels, and validated on
held-out points per cell of the (w0, gamma) plane and per time window.  A
query asks for rho(t) up to a horizon; the network answers it only inside the
box and where every window up to that horizon was within the tolerance in the
query's cell; every other query is propagated by the method itself, which
also judges the error.

The paper contains no such network; it serves parameter scans.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

from . import quapi, workloads

PARAMS = ("w0", "gamma", "lam", "alpha", "eps")


@dataclass
class Box:
    """Parameter ranges around the structured bath.  Toward w0 = 2 with
    lambda = 0.15 the method itself leaves the physical range (|rho| up to 25
    with lags 0..7 of 12 kept exact, 1.8 with 0..11 of 16), its memory far
    shorter than the bath's; over this box it stays within |rho| <= 1."""
    w0: Tuple[float, float] = (0.5, 1.5)
    gamma: Tuple[float, float] = (0.02, 0.1)
    lam: Tuple[float, float] = (0.05, 0.1)
    alpha: Tuple[float, float] = (0.03, 0.07)
    eps: Tuple[float, float] = (0.25, 0.75)

    def lo_hi(self):
        lo = np.array([getattr(self, p)[0] for p in PARAMS])
        hi = np.array([getattr(self, p)[1] for p in PARAMS])
        return lo, hi

    def sample(self, n: int, seed: int) -> np.ndarray:
        lo, hi = self.lo_hi()
        return np.random.default_rng(seed).uniform(lo, hi, (n, len(PARAMS)))

    def contains(self, pts: np.ndarray) -> np.ndarray:
        lo, hi = self.lo_hi()
        return np.all((pts >= lo) & (pts <= hi), axis=1)


@dataclass
class Solver:
    """The method's settings for the trajectories: the structured bath's
    (dk_max 24, lags 0..11 exact, theta 1e-8)."""
    K: int = 24
    n_exact: int = 12
    theta: float = 1e-8
    n_steps: int = 100
    batch: int = 64
    threads: int = 8                         # eta quadratures in parallel (host)

    def solve(self, pts: np.ndarray, progress: bool = False, n_steps: Optional[int] = None) -> np.ndarray:
        """rho(t), t = 0..n_steps (default: the solver's), of every point:
        [n_points][n_steps + 1][2][2], by the batched propagation, `batch` points
        per launch."""
        from concurrent.futures import ThreadPoolExecutor
        n_t = self.n_steps if n_steps is None else n_steps
        base = workloads.structured_bath(n_steps=n_t, K=self.K, n_exact=self.n_exact, theta=self.theta)
        out = np.zeros((len(pts), n_t + 1, 2, 2), dtype=np.complex128)

        def eta(pt):
            w0, g, lam, a, _ = pt
            return quapi.quapi_eta(a, base.bath.ohmic_wc, [w0, g, lam], base.beta, base.dt, self.K)

        with ThreadPoolExecutor(self.threads) as ex:
            etas_all = list(ex.map(eta, pts))
        for s in range(0, len(pts), self.batch):
            chunk = pts[s:s + self.batch]
            etas = np.stack(etas_all[s:s + self.batch])
            Hs = np.stack([workloads.tls_hamiltonian(e, 1.0) for e in chunk[:, 4]])
            prop = quapi.BatchPropagator(base.H, base.q, base.dt, self.K, etas, base.rho0, mask=base.mask,
                                         theta=self.theta, max_steps=n_t, H_batch=Hs)
            prop.step(n_t)
            out[s:s + len(chunk)] = np.transpose(prop.rho_all(0, n_t + 1), (1, 0, 2, 3))
            prop.close()
            if progress:
                print(f"[solver] points {s + len(chunk)} of {len(pts)}", flush=True)
        return out


def free_evolution(pts: np.ndarray, n_t: int, dt: float, rho0: np.ndarray) -> np.ndarray:
    """U(t) rho0 U(t)^+ of the system alone, U = exp(-i H_S t), H_S = (eps/2)
    sigma_z + (1/2) sigma_x, t = 0, dt, ..., (n_t - 1) dt: [n][n_t][2][2]."""
    eps = np.asarray(pts)[:, 4]
    om = np.sqrt(eps ** 2 + 1.0)                     # level splitting
    t = dt * np.arange(n_t)
    ph = 0.5 * om[:, None] * t[None, :]
    c, s = np.cos(ph), np.sin(ph)
    nz, nx = (eps / om)[:, None], (1.0 / om)[:, None]
    # U = cos(ph) 1 - i sin(ph) (nz sigma_z + nx sigma_x)
    U = np.empty((len(eps), n_t, 2, 2), dtype=np.complex128)
    U[..., 0, 0] = c - 1j * s * nz
    U[..., 1, 1] = c + 1j * s * nz
    U[..., 0, 1] = -1j * s * nx
    U[..., 1, 0] = -1j * s * nx
    return U @ rho0 @ np.conj(np.swapaxes(U, -1, -2))


def rho_components(rho: np.ndarray) -> np.ndarray:
    """[..., 2, 2] complex -> [..., 4] real: rho_00, Re rho_01, Im rho_01, rho_11."""
    return np.stack([rho[..., 0, 0].real, rho[..., 0, 1].real, rho[..., 0, 1].imag, rho[..., 1, 1].real], axis=-1)


@dataclass
class Surrogate:
    box: Box = field(default_factory=Box)
    solver: Solver = field(default_factory=Solver)
    width: int = 256
    depth: int = 4
    tol: float = 1e-3
    cells: Tuple[int, int] = (4, 3)          # bins of w0 and gamma for the validation
    windows: int = 5                         # equal time windows of 0..n_steps for the validation
    seed: int = 1
    net: Optional[quapi.MLP] = None
    accepted: Optional[np.ndarray] = None    # [cells w0][cells gamma][windows] bool
    cell_error: Optional[np.ndarray] = None  # held-out error per cell and window (nan: no point)
    history: Dict[str, list] = field(default_factory=dict)
    stream: object = None                    # torch stream of the network and of its batches
    residual: bool = True                    # learn rho(t) minus the system's own evolution
    time_features: bool = True               # add cos/sin of Omega t and w0 t to the inputs

    def _stream(self):
        """One torch stream for the network and the tensor work around it (torch's
        default stream has the null handle, which the library would replace by a
        stream of its own, unordered with torch's)."""
        import torch
        if self.stream is None:
            self.stream = torch.cuda.Stream()
        return self.stream

    # ---- features
    @property
    def n_features(self) -> int:
        return 10 if self.time_features else 6

    def _features(self, pts: np.ndarray, n_t: int) -> np.ndarray:
        """[n_points][n_t][n_features] in [-1, 1]: the parameters and the time,
        then (time_features) cos and sin of Omega t and of w0 t, Omega =
        sqrt(eps^2 + Delta^2) the splitting of H_S and w0 the bath peak: over
        hundreds of steps rho(t) oscillates many times, which a network with
        the time as one input learns poorly.  They are fixed functions of the
        same six inputs."""
        lo, hi = self.box.lo_hi()
        p = 2.0 * (pts - lo) / (hi - lo) - 1.0
        tt = 2.0 * np.arange(n_t) / max(self.solver.n_steps, 1) - 1.0
        f = np.empty((len(pts), n_t, self.n_features), dtype=np.float32)
        f[:, :, :5] = p[:, None, :]
        f[:, :, 5] = tt[None, :]
        if self.time_features:
            t = workloads.structured_bath().dt * np.arange(n_t)
            om = np.sqrt(np.asarray(pts)[:, 4] ** 2 + 1.0)
            w0 = np.asarray(pts)[:, 0]
            f[:, :, 6] = np.cos(om[:, None] * t[None, :])
            f[:, :, 7] = np.sin(om[:, None] * t[None, :])
            f[:, :, 8] = np.cos(w0[:, None] * t[None, :])
            f[:, :, 9] = np.sin(w0[:, None] * t[None, :])
        return f

    def _baseline(self, pts: np.ndarray, n_t: int) -> np.ndarray:
        base = workloads.structured_bath()
        if not self.residual:
            return np.zeros((len(pts), n_t, 2, 2), dtype=np.complex128)
        return free_evolution(pts, n_t, base.dt, base.rho0)

    def _cell(self, pts: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        lo, hi = self.box.lo_hi()
        u = (pts[:, :2] - lo[:2]) / (hi[:2] - lo[:2])
        cw = np.clip((u[:, 0] * self.cells[0]).astype(int), 0, self.cells[0] - 1)
        cg = np.clip((u[:, 1] * self.cells[1]).astype(int), 0, self.cells[1] - 1)
        return cw, cg

    # ---- training and validation
    def fit(self, train_pts: np.ndarray, train_rho: np.ndarray, steps: int = 4000, batch: int = 8192,
            lr: float = 1e-3, lr_final: float = 1e-5, log_every: int = 500):
        """Adam on random mini-batches of (point, t) samples, with the learning
        rate decaying geometrically from lr to lr_final."""
        import torch
        st = self._stream()
        n_t = train_rho.shape[1]
        target = train_rho - self._baseline(train_pts, n_t)
        with torch.cuda.stream(st):
            x = torch.as_tensor(self._features(train_pts, n_t).reshape(-1, self.n_features), device="cuda")
            y = torch.as_tensor(rho_components(target).reshape(-1, 4).astype(np.float32), device="cuda")
            n = x.shape[0]
            batch = min(batch, n)
            if self.net is None:
                self.net = quapi.MLP(self.n_features, self.width, self.depth, 4, max_batch=max(batch, 65536),
                                     seed=self.seed,
                                     stream=st.cuda_stream)
            g = torch.Generator(device="cuda")
            g.manual_seed(self.seed)
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            self.history["loss"] = []
            for s in range(steps):
                idx = torch.randint(0, n, (batch,), device="cuda", generator=g)
                xb, yb = x[idx].contiguous(), y[idx].contiguous()
                self.net.backward(xb, yb, loss)
                self.net.adam(lr * (lr_final / lr) ** (s / max(steps - 1, 1)))
                if log_every and (s % log_every == 0 or s == steps - 1):
                    self.net.sync()
                    self.history["loss"].append((s, loss.item()))
        self.net.sync()

    def predict(self, pts: np.ndarray, n_t: Optional[int] = None) -> np.ndarray:
        """The network's rho(t), t = 0..n_t-1, of every point: [n][n_t][2][2]."""
        import torch
        n_t = self.solver.n_steps + 1 if n_t is None else n_t
        f = self._features(pts, n_t).reshape(-1, self.n_features)
        out = np.empty((f.shape[0], 4), dtype=np.float32)
        step = self.net.max_batch
        with torch.cuda.stream(self._stream()):
            for s in range(0, f.shape[0], step):
                xb = torch.as_tensor(f[s:s + step], device="cuda")
                yb = torch.empty((xb.shape[0], 4), dtype=torch.float32, device="cuda")
                self.net.forward(xb, yb)
                self.net.sync()
                out[s:s + step] = yb.cpu().numpy()
        c = out.reshape(len(pts), n_t, 4).astype(np.float64)
        rho = np.empty((len(pts), n_t, 2, 2), dtype=np.complex128)
        rho[..., 0, 0] = c[..., 0]
        rho[..., 0, 1] = c[..., 1] + 1j * c[..., 2]
        rho[..., 1, 0] = c[..., 1] - 1j * c[..., 2]
        rho[..., 1, 1] = c[..., 3]
        return rho + self._baseline(pts, n_t)

    def _window(self, t: np.ndarray) -> np.ndarray:
        """Time window of step t (0..n_steps): equal spans, the last one closed."""
        n = max(self.solver.n_steps, 1)
        return np.minimum((np.asarray(t) * self.windows) // n, self.windows - 1)

    def validate(self, pts: np.ndarray, rho: np.ndarray) -> np.ndarray:
        """Held-out error of every point (max over t and elements of |rho_net -
        rho_method|); a (cell, window) is accepted when its held-out points are
        all within the tolerance over the window's steps."""
        e_t = np.abs(self.predict(pts, rho.shape[1]) - rho).max(axis=(2, 3))      # [points][t]
        win = self._window(np.arange(rho.shape[1]))
        e_w = np.stack([e_t[:, win == w].max(axis=1) for w in range(self.windows)], axis=1)
        cw, cg = self._cell(pts)
        self.cell_error = np.full(self.cells + (self.windows,), np.nan)
        for a in range(self.cells[0]):
            for b in range(self.cells[1]):
                sel = (cw == a) & (cg == b)
                if sel.any():
                    self.cell_error[a, b] = e_w[sel].max(axis=0)
        self.accepted = np.nan_to_num(self.cell_error, nan=np.inf) <= self.tol
        return e_t.max(axis=1)

    def answers(self, pts: np.ndarray, t_max: int) -> np.ndarray:
        """Which points the network answers up to step t_max: inside the box,
        and every window through t_max's accepted in the point's cell."""
        use = self.box.contains(pts)
        if self.accepted is None:
            return np.zeros(len(pts), dtype=bool)
        cw, cg = self._cell(pts)
        last = int(self._window(np.array([t_max]))[0])
        return use & self.accepted[cw, cg, :last + 1].all(axis=1)

    # ---- queries
    def query(self, pts: np.ndarray, t_max: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
        """rho(t), t = 0..t_max (default n_steps), of every point, and which were
        answered by the network (the rest by the method, propagated to t_max)."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, len(PARAMS))
        t_max = self.solver.n_steps if t_max is None else int(t_max)
        if not 0 <= t_max <= self.solver.n_steps:
            raise ValueError(f"t_max {t_max} outside 0..{self.solver.n_steps}")
        use = self.answers(pts, t_max)
        out = np.empty((len(pts), t_max + 1, 2, 2), dtype=np.complex128)
        if use.any():
            out[use] = self.predict(pts[use], t_max + 1)
        if (~use).any():
            out[~use] = self.solver.solve(pts[~use], n_steps=t_max)
        return out, use


def main(argv=None):
    """Train and validate at a given scale; one JSON line of results.

        python -m paper_2506_03127_amd.surrogate --points 4096 --steps 500   (needs the GPU)
    """
    import argparse
    import json
    import time

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--points", type=int, default=4096, help="training points")
    ap.add_argument("--held-out", type=int, default=512, help="validation points")
    ap.add_argument("--steps", type=int, default=500, help="time steps per trajectory")
    ap.add_argument("--train-steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args(argv)

    import torch
    # torch's device first, before the library's first HIP call (the network
    # and its batches run on a torch stream)
    if not torch.cuda.is_available():
        raise SystemExit("the surrogate needs a GPU")
    sur = Surrogate(solver=Solver(n_steps=args.steps), tol=args.tol)
    sur._stream()
    pts = sur.box.sample(args.points + args.held_out, seed=args.seed)
    t0 = time.perf_counter()
    rho = sur.solver.solve(pts, progress=True)
    t_solve = time.perf_counter() - t0
    train, held = slice(0, args.points), slice(args.points, None)
    t0 = time.perf_counter()
    sur.fit(pts[train], rho[train], steps=args.train_steps, batch=args.batch,
            log_every=max(args.train_steps // 10, 1))
    t_fit = time.perf_counter() - t0
    print(f"[surrogate] loss {sur.history['loss'][0][1]:.3e} -> {sur.history['loss'][-1][1]:.3e}", flush=True)
    err = sur.validate(pts[held], rho[held])
    q = pts[held][:64]
    t0 = time.perf_counter()
    sur.predict(q)
    t_net = time.perf_counter() - t0
    t0 = time.perf_counter()
    sur.solver.solve(q)
    t_method = time.perf_counter() - t0
    out = {
        "points": args.points, "held_out": args.held_out, "time_steps": args.steps,
        "train_steps": args.train_steps, "batch": args.batch,
        "solve_s": t_solve, "fit_s": t_fit, "loss_final": sur.history["loss"][-1][1],
        "held_out_error_median": float(np.median(err)), "held_out_error_p90": float(np.percentile(err, 90)),
        "held_out_error_max": float(err.max()), "tol": args.tol,
        "cells_accepted": int(sur.accepted.all(axis=2).sum()), "cells": int(sur.accepted[..., 0].size),
        "windows": sur.windows,
        "cell_windows_accepted_from_t0": [int(sur.accepted[..., :w + 1].all(axis=2).sum())
                                          for w in range(sur.windows)],
        "query_64_points_network_ms": 1e3 * t_net, "query_64_points_method_ms": 1e3 * t_method,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
