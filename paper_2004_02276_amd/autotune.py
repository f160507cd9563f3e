"""Tile-shape autotuner for the fused right-hand-side kernel.

For a problem (or a size class of problems) it times every compiled tile
shape (tile_x, tile_y) and a set of z-chunk depths kz with HIP events
(`cdns_time_phases`) and keeps the one with the shortest step: the time
per RK step of the phases the tiling changes, the fused right-hand side
(which does the stage update in the default 64x4 tile) plus the separate
update and force kernels (launched in the other tiles, or with bulk
forcing), each as mean launch time x launches per step.  Results are cached in a JSON table keyed by device name,
precision and size class, so the serving loop and the benchmark reuse them.
Tile shape never changes results beyond the rounding of the forcing sum.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

TILES = [(64, 4), (64, 8), (32, 8), (64, 2), (128, 2)]
KZS = [4, 8, 16, 32]


def size_class(pr) -> str:
    """Bucket by point count (powers of two) and aspect (nx >= 64 or not);
    scheme orders other than the default (4, 5) form classes of their own."""
    n = pr.nx * pr.ny * pr.nz
    b = max(0, int(n).bit_length() - 1)
    co, wo = orders(pr)
    scheme = "" if (co, wo) == (4, 5) else f"-c{co}w{wo}"
    return f"2^{b}-{'wide' if pr.nx >= 64 else 'narrow'}{scheme}"


def orders(pr) -> Tuple[int, int]:
    return int(getattr(pr, "central_order", 4)), int(getattr(pr, "weno_order", 5))


def _key(device: str, precision: int, cls: str) -> str:
    return f"{device}|{'fp64' if precision == 0 else 'fp32flux'}|{cls}"


def load_cache() -> Dict:
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(tab: Dict) -> None:
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(tab, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


TILED_PHASES = ("rhs", "rk", "force")


def step_ms(phases: Dict, steps: int) -> float:
    """Per-step time (ms) of the phases the tiling changes, from
    Solver.time_phases output {phase: (mean ms per launch, launches)}."""
    return sum(phases[k][0] * phases[k][1] for k in TILED_PHASES if k in phases) / steps


def tune(pr, precision: int = 0, steps: int = 2, tiles=TILES, kzs=KZS,
         fixed_tile: Optional[Tuple[int, int]] = None, verbose: bool = False,
         save: bool = True) -> Dict:
    """Time every (tile, kz) on `pr`; return {"tile": (tx, ty), "kz": kz,
    "ms": per-step time of the tiled phases, "all": {config: ms}}."""
    import torch

    from .solver import Solver

    dev = torch.cuda.get_device_name(0)
    results = {}
    cand_tiles = [fixed_tile] if fixed_tile else tiles
    if orders(pr)[0] != 4:
        cand_tiles = [(64, 4)]  # the only tile compiled for central orders 2 and 6
    for (tx, ty) in cand_tiles:
        for kz in kzs:
            if kz > pr.nz:
                continue
            s = Solver(pr, precision=precision, tiling=(tx, ty, kz))
            s.time_phases(1, cfl=pr.cfl)  # first launches (code loading) untimed
            s.set_state(pr.w0)
            ph = s.time_phases(steps, cfl=pr.cfl)
            s.close()
            results[f"{tx}x{ty}/kz{kz}"] = step_ms(ph, steps)
            if verbose:
                print(f"  tile {tx}x{ty} kz {kz}: {results[f'{tx}x{ty}/kz{kz}']:.4f} ms per step",
                      flush=True)
    best = min(results, key=results.get)
    t, kz = best.split("/kz")
    tx, ty = (int(v) for v in t.split("x"))
    out = {"tile": [tx, ty], "kz": int(kz), "ms": results[best], "all": results, "device": dev}
    if save:
        tab = load_cache()
        tab[_key(dev, precision, size_class(pr))] = out
        save_cache(tab)
    return out


def lookup(pr, precision: int = 0, device: Optional[str] = None,
           fixed_tile: Optional[Tuple[int, int]] = None) -> Tuple[int, int, int]:
    """Tiling for `pr` from the cache (nearest size class of the same device),
    else the library default shape with a kz giving at least ~1000 blocks."""
    tab = load_cache()
    if device is None:
        try:
            import torch
            device = torch.cuda.get_device_name(0)
        except Exception:
            device = ""
    ent = tab.get(_key(device, precision, size_class(pr)))
    if ent and (fixed_tile is None or tuple(ent["tile"]) == tuple(fixed_tile)):
        return ent["tile"][0], ent["tile"][1], ent["kz"]
    tx, ty = fixed_tile or (64, 4)
    if orders(pr)[0] != 4:
        tx, ty = 64, 4
    tiles = -(-pr.nx // tx) * -(-pr.ny // ty)
    kz = 16
    while kz > 4 and tiles * -(-pr.nz // kz) < 1024:
        kz //= 2
    return tx, ty, kz
