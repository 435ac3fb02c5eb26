"""Convenience layer over the binding: upload a seeded ``workloads.Batch`` into device tensors in the
plan's I/O precision, run the predictor through the C ABI, and return the outputs as host arrays.
Argument marshalling only; all arithmetic happens in libstp.so."""
from __future__ import annotations

import numpy as np
import torch

from . import stp
from . import workloads as W
from .workloads import GENERIC


def io_dtype(prec):
    return torch.float64 if prec == stp.FP64 else torch.float32


def class_of(b, flags_extra=0):
    flags = flags_extra
    if b.physics == GENERIC:
        if b.A is not None:
            flags |= stp.A_PRESENT
        if b.coef_per_element:
            flags |= stp.COEF_PER_ELEMENT
    elif b.coef_per_element:
        flags |= stp.PARAM_PER_ELEMENT
    if b.src is not None:
        flags |= stp.SRC_POINT
    return (b.N, b.m, b.physics, flags)


class DeviceBatch:
    """Device tensors for one uniform batch (inputs uploaded once, outputs allocated)."""

    def __init__(self, plan, b, device="cuda", favg_sum=False):
        dt = io_dtype(plan.prec)
        self.b = b
        n = b.N + 1
        E = b.nelem
        up = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        self.Q = up(b.Q)
        self.params = up(b.params)
        self.A = up(W.coef_abi(b.A, b.coef_per_element))
        self.B = up(W.coef_abi(b.B, b.coef_per_element))
        self.src = up(b.src)
        self.qavg = torch.empty((E, n ** 3, b.m), device=device, dtype=dt)
        self.favg = torch.empty((E, n ** 3, b.m) if favg_sum else (E, 3, n ** 3, b.m), device=device, dtype=dt)
        self.qface = torch.empty((E, 6, n * n, b.m), device=device, dtype=dt)
        self.fface = torch.empty((E, 6, n * n, b.m), device=device, dtype=dt) if b.A is not None else None
        uniform_dt = E == 0 or (np.all(b.dt == b.dt[0]) and np.all(b.h == b.h[0]))
        if uniform_dt:
            self.dt, self.h = (float(b.dt[0]), float(b.h[0])) if E else (0.0, 1.0)
        else:
            self.dt = torch.from_numpy(b.dt).to(device=device, dtype=torch.float64)
            self.h = torch.from_numpy(b.h).to(device=device, dtype=torch.float64)
        self.cbatch = plan.batch(E, self.Q, self.qavg, self.favg, self.qface, self.dt, self.h, params=self.params,
                                 A=self.A, B=self.B, src=self.src, fface=self.fface)

    def clear_outputs(self, value=0.0):
        for t in (self.qavg, self.favg, self.qface, self.fface):
            if t is not None:
                t.fill_(value)

    def outputs(self):
        out = {"qavg": self.qavg, "favg": self.favg, "qface": self.qface}
        if self.fface is not None:
            out["fface"] = self.fface
        return {k: v.double().cpu().numpy() for k, v in out.items()}


def run(plan, b, stream=None, favg_sum=False):
    db = DeviceBatch(plan, b, favg_sum=favg_sum)
    plan.run(db.cbatch, stream)
    torch.cuda.synchronize()
    return db.outputs()


def rounded(b, prec):
    """The batch with every floating input rounded to the I/O precision (the oracle then runs on these)."""
    if prec == stp.FP64:
        return b
    import copy
    r = copy.copy(b)
    f = lambda a: None if a is None else a.astype(np.float32).astype(np.float64)
    r.Q, r.params, r.A, r.B, r.src = f(b.Q), f(b.params), f(b.A), f(b.B), f(b.src)
    return r
