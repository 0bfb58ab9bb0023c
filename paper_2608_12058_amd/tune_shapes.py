"""Pass-shape sweep behind the complex64 pass plans (one GPU).

Times single hypercube passes through qw_time_pass_c64 (fixed coefficients,
caller buffers) and prints two tables:

  rows   ADD passes of one flipped group with L contiguous low bits per row
         (rows of 8 * 2^L bytes), the same 24 bytes per amplitude each: what
         the row length of a strided pass costs;
  plans  every three-orientation plan of n bits (a contiguous group of 12-14
         bits and two high groups of 6-10 bits), each pass in every tile shape
         the kernels have, ranked by the time of one term of the fused
         schedule: the ADD pass of the middle orientation plus half of each end
         orientation's fused pass.
  g0     (--g0-sweep) one group of 8 flipped bits moved up the index, g0 = L ..
         n - 8, in the two shapes the 28-qubit plan uses (2^13 tiles with 512
         threads and 256-byte rows, 2^14 tiles with 1024 threads and 512-byte
         rows), ADD and on-the-fly FUSED: how the rate of a strided pass
         depends on how far apart its rows lie (the rows of one tile fall in
         2^(number of group bits >= 18) different 2 MB blocks of a complex64
         vector).

    python -m paper_2608_12058_amd.tune_shapes --n 28 [--no-rows] [--reps 6]
    python -m paper_2608_12058_amd.tune_shapes --n 28 --g0-sweep [--g0 12,16,20] [--reps 1]
"""
from __future__ import annotations

import argparse
import ctypes
import itertools
import json

SHAPES = [(12, 1024), (13, 1024), (13, 512), (14, 1024)]
OTF_SHAPES = [(13, 512), (14, 1024)]
START, ADD, FUSED = 0, 1, 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--reps", type=int, default=6)
    ap.add_argument("--no-rows", action="store_true")
    ap.add_argument("--no-plans", action="store_true")
    ap.add_argument("--stored-diag", action="store_true", help="also time fused passes that read a stored diagonal")
    ap.add_argument("--g0-sweep", action="store_true", help="only the table of one 8-bit group at every offset g0")
    ap.add_argument("--g0", default="", help="comma-separated offsets for --g0-sweep (default: all)")
    args = ap.parse_args()
    import torch
    import paper_2608_12058_amd as qw
    lib = qw.lib()
    vp = ctypes.c_void_p
    lib.qw_time_pass_c64.argtypes = [ctypes.c_int] * 9 + [vp] * 6 + [vp, ctypes.c_size_t, vp]
    n = args.n
    N = 1 << n
    b1 = torch.zeros(N, dtype=torch.complex64, device="cuda")
    acc = torch.zeros_like(b1)
    psi = torch.zeros_like(b1)
    d = torch.zeros(N if args.stored_diag else 1, dtype=torch.float32, device="cuda")
    ws = qw.Workspace.for_problem(n, 64, True)
    stream = torch.cuda.current_stream()

    def timed(mode, tb, nt, otf, L, g0, h, xcd):
        call = lambda: lib.qw_time_pass_c64(n, mode, tb, nt, otf, L, g0, h, xcd, vp(b1.data_ptr()),
                                            vp(acc.data_ptr()), vp(acc.data_ptr()), vp(b1.data_ptr()),
                                            vp(psi.data_ptr()), vp(d.data_ptr()), vp(ws.ptr()), ws.nbytes,
                                            vp(stream.cuda_stream))
        for _ in range(2):
            qw._check(call())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            call()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / args.reps * 1e3

    print(f"# pass-shape sweep, n = {n} (complex64, streaming loads and stores), microseconds per pass\n")
    if args.g0_sweep:
        # (mode, tile bits, threads, on the fly, passenger bits L, bytes per amplitude)
        kinds = ((ADD, 13, 512, 0, 5, 24), (ADD, 14, 1024, 0, 6, 24), (FUSED, 13, 512, 1, 5, 40),
                 (FUSED, 14, 1024, 1, 6, 40))
        want = [int(x) for x in args.g0.split(",") if x.strip()]
        print("| pass | tile | threads | L | g0 | 2 MB blocks per tile | tile order | us | TB/s moved |")
        print("|---|---|---|---|---|---|---|---|---|")
        for mode, tb, nt, otf, L, bpa in kinds:
            h = tb - L
            for g0 in range(L, n - h + 1):
                if want and g0 not in want:
                    continue
                for xcd in (0, 1):
                    us = timed(mode, tb, nt, otf, L, g0, h, xcd)
                    blocks = 1 << max(0, g0 + h - max(g0, 18))   # group bits at or above bit 18
                    print(f"| {'add' if mode == ADD else 'fused rebuilt'} | 2^{tb} | {nt} | {L} | {g0} | {blocks} | "
                          f"{'XCD-major' if xcd else 'launch'} | {us:.1f} | {bpa * N / us / 1e6:.2f} |", flush=True)
        return
    if not args.no_rows:
        print("| tile | threads | L | row bytes | flipped bits | us | TB/s at 24 B/amp |\n|---|---|---|---|---|---|---|")
        for tb, nt in ((12, 1024), (13, 1024), (14, 1024)):
            g0 = 14 if tb == 14 else 12
            for L in range(1 if tb == 14 else 2, 8):
                h = tb - L
                if h < 1 or g0 + h > n or L >= tb:
                    continue
                us = timed(ADD, tb, nt, 0, L, g0, h, 1)
                print(f"| 2^{tb} | {nt} | {L} | {8 << L} | {g0}..{g0 + h - 1} | {us:.1f} | {24 * N / us / 1e6:.2f} |",
                      flush=True)
        print()
    if args.no_plans:
        return
    fused_kinds = [(1, OTF_SHAPES)] + ([(0, SHAPES)] if args.stored_diag else [])
    best = {}

    def record(key, us, desc):
        if key not in best or us < best[key][0]:
            best[key] = (us, desc)

    groups = set()
    for a in (12, 13, 14):
        for h1 in range(6, 11):
            h2 = n - a - h1
            if 6 <= h2 <= 10:
                groups.add((0, a))
                groups.add((a, h1))
                groups.add((a + h1, h2))
    for g0, h in sorted(groups):
        for (tb, nt), xcd in itertools.product(SHAPES, (0, 1)):
            L = 0 if g0 == 0 else tb - h
            if (g0 == 0 and tb != h) or (g0 > 0 and (L < 4 or g0 < L)):
                continue
            record((g0, h, "add"), timed(ADD, tb, nt, 0, L, g0, h, xcd), f"add {tb}/{nt} L{L} x{xcd}")
            for otf, shapes in fused_kinds:
                if (tb, nt) in shapes:
                    us = timed(FUSED, tb, nt, otf, L, g0, h, xcd)
                    record((g0, h, "fused"), us, f"fused {'rebuilt' if otf else 'stored'} {tb}/{nt} L{L} x{xcd}")
    fused_us = {k: v[0] for k, v in best.items() if k[2] == "fused"}
    plans = []
    for a in (12, 13, 14):
        for h1 in range(6, 11):
            h2 = n - a - h1
            if not 6 <= h2 <= 10:
                continue
            ors = [(0, a), (a, h1), (a + h1, h2)]
            for mid in range(3):
                ends = [o for i, o in enumerate(ors) if i != mid]
                if (*ors[mid], "add") not in best or any((*e, "fused") not in fused_us for e in ends):
                    continue
                t = best[(*ors[mid], "add")][0] + sum(fused_us[(*e, "fused")] for e in ends) / 2
                plans.append((t, ors, mid, best[(*ors[mid], "add")][1], [best[(*e, "fused")][1] for e in ends]))
    plans.sort()
    print("| us per term | orientations (g0, bits) | middle (add every term) | ends (fused every other term) |")
    print("|---|---|---|---|")
    for t, ors, mid, ma, fe in plans[:10]:
        ends = [o for i, o in enumerate(ors) if i != mid]
        print(f"| {t:.1f} | {ors} | {ors[mid]}: {ma} ({best[(*ors[mid], 'add')][0]:.0f} us) | "
              + "; ".join(f"{e}: {f} ({fused_us[(*e, 'fused')]:.0f} us)" for e, f in zip(ends, fe)) + " |")
    print("\nJSON " + json.dumps({"n": n, "best_plan": {"us_per_term": plans[0][0], "orientations": plans[0][1],
                                                        "middle": plans[0][2]} if plans else None}))


if __name__ == "__main__":
    main()
