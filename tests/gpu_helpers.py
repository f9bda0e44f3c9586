"""Shared helpers of the GPU parity tests: device copies of seeded inputs,
oracle expectations, and the comparison bar.

The bar: counts, element counts and materialised map outputs bit-exact; max
equal as a float (+0 and -0 compare equal); FP64 sums within 1e-6 relative
error of the FP64 oracle (a zero reference requires an exact zero).
"""
from __future__ import annotations

import numpy as np
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc

REL_TOL = 1e-6


def dev(a: np.ndarray | None, offset: int = 0) -> torch.Tensor | None:
    """Device copy of a float32 array, optionally starting `offset` floats into
    a larger allocation (to exercise unaligned base pointers)."""
    if a is None:
        return None
    buf = torch.empty(a.size + offset + 4, dtype=torch.float32, device="cuda")
    view = buf[offset:offset + a.size]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return view


def oracle_result(p: datagen.Part) -> oracle.Result:
    return oracle.run_task(p.kid, p.ops, p.n, p.x, p.y, seed=p.seed, pid=p.pid,
                           coef=p.coef, c=p.c)


class DevParts:
    """Device copies of a list of partitions and their sparkcl tasks."""

    def __init__(self, parts, xoff: int = 0, yoff: int = 0, out: bool = False):
        self.parts = parts
        self.keep = []
        self.outs = []
        self.tasks = []
        for p in parts:
            x = dev(p.x, xoff) if p.x is not None else None
            y = dev(p.y, yoff) if p.y is not None else None
            o = None
            if out and p.kid != datagen.MC_PI:
                o = torch.full((max(p.n, 1),), float("nan"), dtype=torch.float32,
                               device="cuda")[:p.n]
            self.keep += [x, y]
            self.outs.append(o)
            self.tasks.append(sc.task(p.kid, p.n, x, y, o, ops=p.ops, seed=p.seed,
                                      pid=p.pid, coef=p.coef, c=p.c))


def check_result(g: sc.Result, o: oracle.Result, kid: int, ops: int, where: str = ""):
    assert g.status == 0, where
    assert g.n == o.n, f"{where}: n {g.n} != {o.n}"
    assert g.count == o.count, f"{where}: count {g.count} != {o.count}"
    if ops & datagen.MAX:
        assert np.float32(g.max) == np.float32(o.max), f"{where}: max {g.max} != {o.max}"
    else:
        assert g.max == -np.inf
    if ops & datagen.SUM:
        if o.sum == 0.0:
            assert g.sum == 0.0, f"{where}: sum {g.sum} != 0"
        else:
            rel = abs(g.sum - o.sum) / abs(o.sum)
            assert rel <= REL_TOL, f"{where}: sum {g.sum!r} vs {o.sum!r} rel {rel:.3e}"
    else:
        assert g.sum == 0.0


def check_total(tot: sc.Result, per: list, ops: int):
    o = oracle.rdd_total(per, ops)
    check_result(tot, o, 0, ops, "rdd total")
