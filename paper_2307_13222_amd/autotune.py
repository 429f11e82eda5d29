"""Autotuner for the H*v launch schedules.

Sweeps the schedule knobs of a Hamiltonian (Hubbard T_up kernel: block
tiles with their split, or slabs with their width, workgroups per XCD and
rows per work item; T_dn kernel variant; spin rank-table placement and
workgroups per CU), times w = H v for each candidate with HIP events on the
launch stream, keeps the fastest and records it in a JSON table keyed by
(model kind, dimensions, dtype, block width). Later runs look the key up and
apply the stored schedule without sweeping. Only launch geometry changes:
results agree up to floating-point summation order.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, List, Optional

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "schedules.json")


def schedule_key(ham, dtype: str, nvec: int) -> str:
    b = ham.basis
    m = ham.model
    kind = b.kind
    return f"{kind}:n{b.n_sites}:dim{b.dim}:{getattr(m, 'name', '')}:{dtype}:v{nvec}"


def candidates(ham, quick: bool = False) -> List[Dict[str, int]]:
    """Schedules to time. Hubbard: the block-tile T_up kernel (hub_sweep 7)
    over tile splits (hub_tile_bits: -1 = the fewest top sites whose blocks
    fit LDS, or a few more: smaller blocks, more far hops) and T_dn variants,
    and the slab kernels (hub_sweep 3, 5; slab width, workgroups per XCD,
    rows per item, row order). Spin: the one-pass kernel over placements of
    the rank tables (LDS 32-bit, LDS narrowed, global) x workgroups per CU,
    and the block-staged product over split points (-1 = its own choice).
    Every candidate sets the layout (spin_split), since a schedule keeps
    the fields a candidate leaves out. Candidates the Hamiltonian cannot
    take are skipped when timed."""
    if ham.basis.kind == "hubbard":
        out = []
        bits = (-1, 5) if quick else (-1, 3, 5, 6)
        for tb, rc, g in itertools.product(bits, (6,) if quick else (5, 6), (32,) if quick else (16, 32, 64)):
            out.append({"hub_sweep": 7, "hub_tile_bits": tb, "hub_row_cols": rc, "hub_groups": g})
        slab = itertools.product((128,) if quick else (64, 128), (128,) if quick else (64, 128, 256),
                                 (16,) if quick else (16, 32), (6,) if quick else (5, 6),
                                 (5,) if quick else (3, 5), (2,) if quick else (1, 2))
        for cw, g, rows, rc, sw, ro in slab:
            out.append({"hub_slab_cols": cw, "hub_groups": g, "hub_item_rows": rows, "hub_row_cols": rc,
                        "hub_sweep": sw, "hub_row_order": ro})
        return out
    per = (2, 8) if quick else (1, 2, 4, 8, 16)
    out = [{"spin_split": -1, "spin_tables": t, "spin_per_cu": p} for t in (1, 2, 3) for p in per]
    los = (-1,) if quick else (-1, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17)
    out += [{"spin_split": 2, "spin_blk_lo": lo} for lo in los if lo < ham.basis.n_sites]
    return out


def time_mult(ham, v, w, reps: int = 5) -> float:
    """Median milliseconds of one H*v (HIP events on the current stream)."""
    import torch
    ham.mult(v, w)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ham.mult(v, w)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(ham, dtype: str = "f64", nvec: int = 1, reps: int = 5, cands: Optional[List[Dict]] = None,
         table: str = DEFAULT_TABLE, force: bool = False) -> Dict:
    """Apply the best schedule for this Hamiltonian; sweep if unknown."""
    import torch
    key = schedule_key(ham, dtype, nvec)
    tab = _load(table)
    if key in tab and not force:
        ham.set_schedule(**tab[key]["schedule"])
        return {"key": key, "schedule": tab[key]["schedule"], "ms": tab[key]["ms"], "swept": False}
    tdt = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128, "c64": torch.complex64}[dtype]
    dim = ham.basis.dim
    shape = (dim,) if nvec == 1 else (dim, nvec)
    g = torch.Generator(device="cuda").manual_seed(1)
    v = torch.rand(shape, dtype=torch.float64 if not tdt.is_complex else torch.complex128,
                   device="cuda", generator=g).to(tdt) - 0.5
    w = torch.empty_like(v)
    from .api import HphiError
    results = []
    for c in (cands or candidates(ham)):
        try:
            ham.set_schedule(**c)
            results.append((time_mult(ham, v, w, reps), c))
        except HphiError:
            continue      # a schedule this Hamiltonian or block cannot take
    if not results:
        raise HphiError("autotune: no candidate schedule runs")
    results.sort(key=lambda t: t[0])
    best_ms, best = results[0]
    ham.set_schedule(**best)
    tab[key] = {"schedule": best, "ms": best_ms, "n_candidates": len(results),
                "worst_ms": results[-1][0]}
    os.makedirs(os.path.dirname(table), exist_ok=True)
    tmp = table + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, table)
    del v, w
    return {"key": key, "schedule": best, "ms": best_ms, "swept": True, "n_valid": len(results),
            "table": [(round(t, 4), c) for t, c in results[:8]], "worst_ms": results[-1][0]}
