"""Nuclear-norm proximal gradient for matrix completion, as a client of the
serving loop (section 2: singular value soft-thresholding is the proximal
operator of tau ||.||_*, the subroutine of such methods).

    min_X  f(X) + lam ||X||_*,   f(X) = ||P_Omega(X - M)||_F^2 / 2,
    X_{k+1} = SVT_{eta lam}(X_k - eta P_Omega(X_k - M)),

with eta = 1 (the gradient P_Omega(X - M) is 1-Lipschitz).  The iterates and
the observed data stay on the device; the gradient step is a few elementwise
torch operations on the caller's stream, and every thresholding is one
request to a psvt Server (ordered after that work by the server).  With
``warm`` the sign iteration of step k + 1 may start from step k's (I + S)/2
(psvt.h: psvt_config.warm_pi, fewer iterations).  A warm start keeps the
previous sign for directions whose singular value crossed tau while within
about 1e-3 theta of it, an error in the result of at most the inputs'
change ||G_k - G_{k-1}||_F (the crossing singular values moved at least
|sigma - tau|, and their moves add up to at most that norm, by the
Hoffman-Wielandt inequality).  The loop therefore warm starts only when
that change is at most ``warm_tol`` times ||X_k||_F (the scale of the
result), and starts cold otherwise (early steps, where the iterate still
changes a lot).

``run_loops`` drives many such solvers at once: loops arrive as a Poisson
process, each issues its next step as soon as the previous one is done, and
the driver polls the server for completions (one host thread).
"""
from __future__ import annotations

import time
from typing import List, Optional

import numpy as np


class CompletionLoop:
    """One proximal-gradient solver whose thresholdings go to a server."""

    def __init__(self, M_obs, mask, lam: float, steps: int, eta: float = 1.0, warm: bool = True, name: str = "",
                 warm_tol: float = 5e-3, record_steps=()):
        import torch
        self.torch = torch
        self.M_obs = M_obs            # observed entries (zeros elsewhere), device float32
        self.mask = mask              # 0/1 device float32
        self.lam, self.eta, self.steps, self.warm = float(lam), float(eta), int(steps), bool(warm)
        self.warm_tol = float(warm_tol)
        self.name = name
        self.record_steps = set(record_steps)
        m, n = M_obs.shape
        s = n if n < m else m        # the Gram side (right-sided iff n < m)
        self.pi = torch.empty((s, s), dtype=torch.float32, device=M_obs.device)
        self.reset()

    def reset(self):
        """Back to X = 0 at step 0 (the problem data are kept)."""
        self.X = self.torch.zeros_like(self.M_obs)
        self.pi.zero_()
        self.k = 0
        self.warm_steps = 0
        self.ticket = None
        self.G = self.G_prev = self.Y = None
        self.t_start = None
        # record of (step, G, Y, warm, warm_pi as submitted or None) for checks
        self.inputs: List = []

    @property
    def tau(self) -> float:
        return self.eta * self.lam

    def gradient_step(self):
        """G = X - eta P_Omega(X - M), on the caller's stream."""
        return self.X - self.eta * self.mask * (self.X - self.M_obs)

    def use_warm(self) -> bool:
        """Warm start iff ||G_k - G_{k-1}||_F <= warm_tol ||X_k||_F (a bound
        on the warm start's error in the result; see the module text)."""
        if not self.warm or self.k == 0 or self.G_prev is None:
            return False
        change = float((self.G - self.G_prev).norm().item())
        return change <= self.warm_tol * float(self.X.norm().item())

    def submit(self, srv, record: bool = False):
        self.G_prev = self.G
        self.G = self.gradient_step()
        warm = self.use_warm()
        self.warm_steps += int(warm)
        record = record or self.k in self.record_steps
        snap = self.pi.clone() if (record and warm) else None   # the request overwrites pi
        self.ticket, self.Y = srv.submit(self.G, self.tau, warm_pi=self.pi if warm else None, pi_out=self.pi)
        if record:
            self.inputs.append((self.k, self.G, self.Y, warm, snap))

    def complete(self):
        self.X = self.Y
        self.k += 1
        self.ticket = None
        return self.k >= self.steps

    def objective(self) -> float:
        """f(X) + lam ||X||_* with the nuclear norm from torch's SVD (a
        diagnostic on the caller's side, not part of the path)."""
        torch = self.torch
        r = self.mask * (self.X - self.M_obs)
        nuc = torch.linalg.svdvals(self.X.double()).sum().item()
        return 0.5 * float((r.double() ** 2).sum().item()) + self.lam * nuc


def solve(srv, loop: CompletionLoop, record: bool = False):
    """Run one loop to its last step (blocking), returns its iterate."""
    from . import RQ_DONE
    while True:
        loop.submit(srv, record)
        state = srv.wait(loop.ticket, timeout=600.0)
        if state != RQ_DONE:
            raise RuntimeError("request failed in %s at step %d" % (loop.name, loop.k))
        if loop.complete():
            return loop.X


def run_loops(srv, loops: List[CompletionLoop], arrivals: np.ndarray, poll_s: float = 0.0,
              record_every: int = 0) -> dict:
    """Drive ``loops`` through the server: loop i starts at ``arrivals[i]``
    seconds after the call, and each loop submits its next step as soon as
    its previous one is done (steps in a loop's ``record_steps``, or every
    ``record_every``-th step, are recorded).  Returns counts and the wall
    time."""
    from . import RQ_DONE, RQ_FAILED
    t0 = time.perf_counter()
    pending = sorted(range(len(loops)), key=lambda i: arrivals[i])
    active: List[CompletionLoop] = []
    submitted = failed = 0
    nxt = 0
    while nxt < len(pending) or active:
        now = time.perf_counter() - t0
        while nxt < len(pending) and arrivals[pending[nxt]] <= now:
            lp = loops[pending[nxt]]
            lp.t_start = now
            lp.submit(srv, record_every > 0 and lp.k % record_every == 0)
            submitted += 1
            active.append(lp)
            nxt += 1
        still = []
        for lp in active:
            st = srv.poll(lp.ticket)
            if st == RQ_DONE:
                if not lp.complete():
                    lp.submit(srv, record_every > 0 and lp.k % record_every == 0)
                    submitted += 1
                    still.append(lp)
            elif st == RQ_FAILED:
                failed += 1
            else:
                still.append(lp)
        active = still
        if poll_s:
            time.sleep(poll_s)
    return {"submitted": submitted, "failed": failed, "wall_s": time.perf_counter() - t0}
