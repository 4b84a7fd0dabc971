"""Benchmark: 2048-bit Paillier enc+dec throughput of the hot path on one MI355X.

Workload (the paper-like configuration): a 2048-bit key (n^2 of 4096 bits),
8 simulated edge nodes each holding a 65536-dim float64 vector ~ N(0,1),
quantized with scale 2^20 and offset 2^23.  One step runs the whole hot path
over that batch:

    quantize (8 x 65536) -> encrypt (524288) -> 8-way homomorphic sum (65536)
    -> CRT decrypt (65536) -> dequantize with weight 8 (65536)

`value` = (encryptions + decryptions) per second of the batched path (one
launch per phase over all nodes), inputs resident in HBM.  The plain path
(one launch per call and node, synchronised after every call) is timed on the
same data and reported beside it.  One JSON line is printed.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NBITS = 2048
NODES = 8
LENGTH = 65536
CONFIG_SEED = 2
# MI355X: 256 CUs x 4 SIMD x 16 lanes, one v_mad_u64_u32 (32x32->64 product
# with 64-bit accumulate) per lane per clock at 2.4 GHz.
PEAK_PRODUCTS = 256 * 64 * 2.4e9


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def montgomery_products_per_encrypt(nbits_n: int, n: int, window: int) -> tuple[int, int]:
    """Montgomery products in the encryption schedule and the algorithmic
    32x32-bit limb products they stand for (2 S^2 + S with S 32-bit limbs of
    n^2, the textbook CIOS count)."""
    w = window
    nw = (n.bit_length() + w - 1) // w
    digits = [(n >> (i * w)) & ((1 << w) - 1) for i in range(nw)]
    mults = sum(1 for d in digits[:-1] if d != 0)
    mm = 2 + ((1 << w) - 2) + w * (nw - 1) + mults + 1
    S = 2 * ((nbits_n + 31) // 32)
    return mm, mm * (2 * S * S + S)


def montgomery_products_per_decrypt(p: int, q: int, window: int) -> tuple[int, int]:
    """Both CRT halves: REDC + R^3 product + table + powering + conversion."""
    w = window
    total_mm, total_prod = 0, 0
    for s in (p, q):
        e = s - 1
        eb = max((p - 1).bit_length(), (q - 1).bit_length())
        nw = (eb + w - 1) // w
        digits = [(e >> (i * w)) & ((1 << w) - 1) for i in range(nw)]
        mults = nw - 1  # exponents differ per half: every window multiplies
        mm = 1 + 1 + ((1 << w) - 2) + w * (nw - 1) + mults + 1
        S = (s * s).bit_length() + 31 >> 5
        total_mm += mm
        total_prod += mm * (2 * S * S + S)
    return total_mm, total_prod


# ------------------------------------------------------------- CPU baseline
def _oracle_job(args):
    kind, key, a, b = args
    from oracle import paillier as O
    if kind == "enc":
        return O.encrypt(key, a, b)
    return O.decrypt(key, a)


def cpu_baseline(p: int, q: int, ms, rs, cts, budget_s: float = 20.0) -> dict:
    """The oracle as it stands, on every host core, over a bounded sample."""
    from oracle import paillier as O
    cores = len(os.sched_getaffinity(0))
    pk, sk = O.derive_keys(p, q)
    per_core = 6
    n_enc = n_dec = per_core * cores
    jobs = [("enc", pk, ms[i % len(ms)], rs[i % len(rs)]) for i in range(n_enc)]
    jobs += [("dec", sk, cts[i % len(cts)], None) for i in range(n_dec)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_job, jobs, chunksize=1)
    dt = time.perf_counter() - t0
    return {"value": (n_enc + n_dec) / dt, "unit": "ops/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_enc} encryptions + {n_dec} decryptions of the same 2048-bit "
                      f"workload ({dt:.1f} s wall, multiprocessing pool of {cores})"}


# --------------------------------------------------------------------- main
def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--window", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs the hot path on a single MI355X "
              "(see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2601_14980_amd import pc2
    from workload import gen

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    p, q = gen.primes_for(CONFIG_SEED, NBITS)
    n = p * q
    qp = gen.Q_PLAIN
    xs = gen.normal_vectors(CONFIG_SEED, [LENGTH] * NODES)
    rs = [gen.gen_r_limbs(n, LENGTH, NBITS // 32, CONFIG_SEED, extra=k) for k in range(NODES)]
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s")

    ctx = pc2.Context(0)
    if args.window:
        ctx.set_option(pc2.PC2_OPT_WINDOW, args.window)
    ctx.reserve(NBITS)
    sk = pc2.SecretKey(ctx, NBITS, p, q)
    pk = sk.public
    L = sk.L
    total = NODES * LENGTH
    x_all = torch.from_numpy(np.concatenate(xs)).cuda()
    r_all = pc2.to_device_limbs(np.concatenate(rs))
    m_all = torch.empty(total, dtype=torch.int64, device="cuda")
    c_all = torch.empty((total, 2 * L), dtype=torch.int32, device="cuda")
    agg = torch.empty((LENGTH, 2 * L), dtype=torch.int32, device="cuda")
    msum = torch.empty((LENGTH, L), dtype=torch.int32, device="cuda")
    xo = torch.empty(LENGTH, dtype=torch.float64, device="cuda")
    m2_all = m_all.view(torch.int32).reshape(total, 2)
    c_nodes = [c_all[k * LENGTH:(k + 1) * LENGTH] for k in range(NODES)]
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    enc_ms: list[float] = []
    dec_ms: list[float] = []

    def step_batched(record: bool) -> None:
        pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, x_all, m_all)
        ev[0].record(stream)
        pc2.pc2_encrypt(pk, m2_all, r_all, c_all)
        ev[1].record(stream)
        pc2.pc2_hom_sum(pk, c_nodes, agg)
        ev[2].record(stream)
        pc2.pc2_decrypt(sk, agg, msum)
        ev[3].record(stream)
        pc2.pc2_dequantize(ctx, qp.log2_scale, qp.offset, msum, NODES, xo)
        if record:
            torch.cuda.synchronize()
            enc_ms.append(ev[0].elapsed_time(ev[1]))
            dec_ms.append(ev[2].elapsed_time(ev[3]))

    def step_plain() -> None:
        for k in range(NODES):
            sl = slice(k * LENGTH, (k + 1) * LENGTH)
            pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, x_all[sl], m_all[sl])
            ctx.sync()
        for k in range(NODES):
            sl = slice(k * LENGTH, (k + 1) * LENGTH)
            pc2.pc2_encrypt(pk, m2_all[sl], r_all[sl], c_all[sl])
            ctx.sync()
        pc2.pc2_hom_sum(pk, c_nodes, agg)
        ctx.sync()
        pc2.pc2_decrypt(sk, agg, msum)
        ctx.sync()
        pc2.pc2_dequantize(ctx, qp.log2_scale, qp.offset, msum, NODES, xo)
        ctx.sync()

    ops_per_step = total + LENGTH
    for i in range(args.warmup):
        step_batched(record=False)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    status = ctx.sync()
    if status != 0:
        log(f"device reported status {status}")
        return 1
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step_batched(record=True)
        log(f"timed step {i + 1}/{args.steps}: encrypt {enc_ms[-1]:.1f} ms, "
            f"decrypt {dec_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    if ctx.sync() != 0:
        log("device reported a data error in the timed steps")
        return 1
    ms_per_step = 1e3 * elapsed / args.steps
    value = ops_per_step / (elapsed / args.steps)

    # end-to-end integer check on every element of the last step:
    # Dec(prod_k Enc(m_k)) == sum_k m_k
    m_host = m_all.cpu().numpy().view(np.uint64).reshape(NODES, LENGTH)
    sums = m_host.astype(object).sum(axis=0)
    got = pc2.from_device_limbs(msum)
    got_int = got[:, 0].astype(object) + (got[:, 1].astype(object) << 32)
    exact = bool(np.all(got[:, 2:] == 0)) and bool(np.all(got_int == sums))

    # plain path
    t_plain = []
    for i in range(args.plain_steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step_plain()
        t_plain.append(time.perf_counter() - t1)
        log(f"plain step {i + 1}/{args.plain_steps}: {t_plain[-1] * 1e3:.0f} ms")
    plain_value = ops_per_step / (sum(t_plain) / len(t_plain)) if t_plain else None

    w = ctx.get_option(pc2.PC2_OPT_WINDOW) or 5
    mm_enc, prod_enc = montgomery_products_per_encrypt(NBITS, n, w)
    enc_avg_s = sum(enc_ms) / len(enc_ms) / 1e3
    achieved = prod_enc * total / enc_avg_s
    mm_dec, prod_dec = montgomery_products_per_decrypt(p, q, w)

    cpu = None
    if not args.no_cpu_baseline:
        from workload.limbs import ints_from_limbs
        ms_s = [int(v) for v in m_host[0, :64]]
        rs_s = ints_from_limbs(rs[0][:64])
        cts = ints_from_limbs(pc2.from_device_limbs(agg[:64]))
        log("timing the oracle on the host cores")
        cpu = cpu_baseline(p, q, ms_s, rs_s, cts)

    out = {
        "metric": "2048-bit Paillier enc+dec ops/sec, batched vs plain; serving p50/p99 latency",
        "value": round(value, 1),
        "unit": "ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "2048-bit key, 8 nodes x 65536 float64 ~ N(0,1), scale 2^20, "
                               "offset 2^23: quantize, encrypt 524288, 8-way sum, decrypt 65536, "
                               "dequantize", "nbits": NBITS, "nodes": NODES, "length": LENGTH,
                   "window": w, "path": "batched"},
        "enc_per_s": round(total / enc_avg_s, 1),
        "dec_per_s": round(LENGTH / (sum(dec_ms) / len(dec_ms) / 1e3), 1),
        "plain": ({"value": round(plain_value, 1), "unit": "ops/s",
                   "ms_per_step": round(1e3 * sum(t_plain) / len(t_plain), 2)}
                  if t_plain else None),
        "batched_over_plain": round(value / plain_value, 3) if t_plain else None,
        "end_to_end_exact": exact,
        "roofline": {"bound": "alu", "kernel": "k_encrypt",
                     "achieved": round(achieved / 1e12, 3),
                     "peak": round(PEAK_PRODUCTS / 1e12, 3),
                     "unit": "T limb-products/s (32x32->64, v_mad_u64_u32)",
                     "frac": round(achieved / PEAK_PRODUCTS, 4),
                     "traffic": None,
                     "per_launch_products": prod_enc * total,
                     "mm_per_encrypt": mm_enc,
                     "avg_launch_ms": round(enc_avg_s * 1e3, 3)},
        "cpu_baseline": cpu,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0 if exact else 1


if __name__ == "__main__":
    sys.exit(main())
