"""Autotuner for the Jacobi tiles of the batched (and single) solve.

The one-sided Jacobi kernels have two launch-shape parameters per problem of
padded order ``np`` (``n`` rounded up to 64):

* ``kc``: row chunks the Gram matrix of a block pair is summed over (split-K
  of the Gram kernel; a power of two with ``np % (16 kc) == 0``);
* ``rrows``: rows of the block pair one rotation work group updates (a
  multiple of 64 dividing ``np``).

Few large chunks mean fewer partial Gram tiles to reduce and fewer work
groups; many small ones fill the chip when few problems run at once.  The
tuner times the Jacobi phase of a batch of ``per_bucket`` problems of each
order (the batched workload's generator at that size) for every candidate
and keeps the fastest, giving a table of rows ``(np_max, kc, rrows)`` that
``solve_batched(..., tiles=table)`` and ``solve_h1(..., tiles=table)`` take.

``--workload`` instead tunes on the batched workload itself: starting from the
library's built-in choice, coordinate descent over the buckets, each trial
timing the Jacobi phase of the whole 256-problem batch.

Usage::

    python -m paper_2008_08825_amd.tune --out tiles.json            # 64..1024
    python -m paper_2008_08825_amd.tune --nps 64,128 --per-bucket 4
    python -m paper_2008_08825_amd.tune --workload --repeats 3 --out tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

KC_CHOICES = (1, 2, 4, 8, 16, 32)
RROWS_CHOICES = (64, 128, 256)


def candidates(np_: int):
    """Valid (kc, rrows) pairs for padded order ``np_``."""
    if np_ <= 0 or np_ % 64:
        raise ValueError("np must be a positive multiple of 64")
    out = []
    for kc in KC_CHOICES:
        if np_ % (16 * kc):
            continue
        for rr in RROWS_CHOICES:
            if np_ % rr == 0:
                out.append((kc, rr))
    return out


def validate(table):
    """Rows (np_max, kc, rrows) with np_max ascending, kc a power of two, rrows a multiple of 64."""
    last = 0
    for row in table:
        np_max, kc, rr = (int(v) for v in row)
        if np_max <= last or kc < 1 or kc & (kc - 1) or rr < 64 or rr % 64:
            raise ValueError(f"invalid tile row {row}")
        last = np_max
    return [tuple(int(v) for v in row) for row in table]


def save(table, path: str, meta=None):
    with open(path, "w") as f:
        json.dump({"tiles": [list(r) for r in validate(table)], "meta": meta or {}}, f, indent=1)


def load(path: str):
    with open(path) as f:
        return validate(json.load(f)["tiles"])


PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles_gfx950.json")


def packaged():
    """The table ``--workload`` wrote on an MI355X for the 256-problem batch (orders 128..1024)."""
    return load(PACKAGED)


def tune(nps=tuple(range(64, 1025, 64)), precision="mixed", per_bucket=16, repeats=2, seed=0,
         log=None):
    """Time every candidate per bucket; returns (table, report)."""
    import torch

    from . import api, inputs

    dev = torch.device("cuda:0")
    table, report = [], []
    for np_ in nps:
        probs = [inputs.batch_problem(10000 + seed * 1000 + np_ + i, np_) for i in range(per_bucket)]
        As = [torch.from_numpy(a).to(dev) for a, _ in probs]
        Bs = [torch.from_numpy(b).to(dev) for _, b in probs]
        need = max(api.batched_workspace_bytes([np_] * per_bucket, precision=precision,
                                               tiles=[(np_, kc, rr)]) for kc, rr in candidates(np_))
        work = torch.empty(need, dtype=torch.uint8, device=dev)
        best = None
        times = {}
        for kc, rr in candidates(np_):
            tiles = [(np_, kc, rr)]
            ms = []
            for _ in range(repeats):
                _, infos, st = api.solve_batched(As, Bs, precision=precision, tiles=tiles, timing=1,
                                                 work=work, check=False)
                if st != 0:
                    raise RuntimeError(f"status {st} while tuning np={np_}")
                ms.append(infos[0]["ms_phase"][3])  # Jacobi phase of the whole batch
            t = min(ms)
            times[f"{kc}x{rr}"] = round(t, 3)
            if best is None or t < best[0]:
                best = (t, kc, rr)
        table.append((np_, best[1], best[2]))
        report.append({"np": np_, "best": f"{best[1]}x{best[2]}", "jacobi_ms": times})
        if log:
            log(f"np={np_}: best kc={best[1]} rrows={best[2]} ({best[0]:.2f} ms); {times}")
        del As, Bs, work
        torch.cuda.synchronize()
    return validate(table), report


def default_kc(np_: int) -> int:
    """The library's own Gram split for one problem (enough work groups to fill the chip)."""
    pairs, kc = np_ // 64, 1
    while pairs * kc < 1024 and kc * 2 <= np_ // 16 and np_ % (kc * 32) == 0 and kc < 64:
        kc *= 2
    return kc


def builtin_batch_tiles(np_: int):
    """The library's built-in batch choice: Gram row chunks of about 256 rows, largest rotation group."""
    k = 1
    while np_ // (2 * k) >= 256 and np_ % (32 * k) == 0 and 2 * k <= default_kc(np_):
        k *= 2
    rr = 256 if np_ % 256 == 0 else (128 if np_ % 128 == 0 else 64)
    return k, rr


def tune_workload(ns, precision="mixed", repeats=3, log=None):
    """Coordinate descent over the buckets of a real batch of orders ``ns``.

    Starting from the built-in choice, each bucket (largest first) tries every
    candidate with the others fixed, timing the Jacobi phase of the whole batch
    (the problems of all buckets run together in the grouped launches).
    """
    import torch

    from . import api, inputs

    dev = torch.device("cuda:0")
    probs = [inputs.batch_problem(i, n) for i, n in enumerate(ns)]
    As = [torch.from_numpy(a).to(dev) for a, _ in probs]
    Bs = [torch.from_numpy(b).to(dev) for _, b in probs]
    del probs
    buckets = sorted({((n + 63) // 64) * 64 for n in ns})
    cur = {b: builtin_batch_tiles(b) for b in buckets}
    cap = max(kc for b in buckets for kc, _ in candidates(b))
    need = max(api.batched_workspace_bytes(ns, precision=precision, tiles=[(b, min(kc, cap), 64)])
               for b in buckets for kc, _ in candidates(b))
    work = torch.empty(need, dtype=torch.uint8, device=dev)

    def table(c):
        return [(b, *c[b]) for b in buckets]

    def jacobi_ms(c):
        ms = []
        for _ in range(repeats):
            _, infos, st = api.solve_batched(As, Bs, precision=precision, tiles=table(c), timing=1,
                                             work=work, check=False)
            if st != 0:
                raise RuntimeError(f"status {st} while tuning")
            ms.append(infos[0]["ms_phase"][3])
        return min(ms)

    base = best_t = jacobi_ms(cur)
    if log:
        log(f"built-in tiles: Jacobi {base:.2f} ms")
    for b in sorted(buckets, reverse=True):
        for cand in candidates(b):
            if cand == cur[b] or cand[0] > default_kc(b):
                continue
            trial = dict(cur)
            trial[b] = cand
            t = jacobi_ms(trial)
            if t < best_t:
                best_t, cur = t, trial
        if log:
            log(f"np={b}: kc={cur[b][0]} rrows={cur[b][1]}, batch Jacobi {best_t:.2f} ms")
    return validate(table(cur)), {"builtin_ms": round(base, 3), "tuned_ms": round(best_t, 3)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--nps", default="", help="comma-separated padded orders (default 64..1024)")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--per-bucket", type=int, default=16)
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--out", default="")
    ap.add_argument("--workload", action="store_true",
                    help="tune on the 256-problem batched workload itself (coordinate descent)")
    args = ap.parse_args()
    nps = tuple(int(v) for v in args.nps.split(",")) if args.nps else tuple(range(64, 1025, 64))
    t0 = time.time()
    if args.workload:
        from . import inputs

        table, report = tune_workload(inputs.batch_sizes(), args.precision, max(args.repeats, 1),
                                      log=lambda m: print(m, flush=True))
        meta = {"precision": args.precision, "mode": "workload (256 problems, n in [64, 1024], seed 0)",
                "seconds": round(time.time() - t0, 1), "report": report}
    else:
        table, report = tune(nps, args.precision, args.per_bucket, args.repeats,
                             log=lambda m: print(m, flush=True))
        meta = {"precision": args.precision, "per_bucket": args.per_bucket,
                "seconds": round(time.time() - t0, 1), "report": report}
    if args.out:
        save(table, args.out, meta)
    print(json.dumps({"tiles": table}))


if __name__ == "__main__":
    main()
