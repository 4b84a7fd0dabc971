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
import ctypes
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


def sliding_schedule(e: int, w: int) -> list[tuple[int, int]]:
    """Left-to-right sliding windows of e: (squarings, odd digit or 0) per
    entry, the first entry's digit being the starting power (the schedule
    the kernels run for a wave-uniform exponent)."""
    out, sq, i, first = [], 0, e.bit_length() - 1, True
    while i >= 0:
        if not (e >> i) & 1:
            sq += 1
            i -= 1
            continue
        j = max(i - w + 1, 0)
        while not (e >> j) & 1:
            j += 1
        d = (e >> j) & ((1 << (i - j + 1)) - 1)
        out.append((0 if first else sq + i - j + 1, d))
        first, sq, i = False, 0, j - 1
    if sq:
        out.append((sq, 0))
    return out


def schedule_products(e: int, w: int) -> int:
    """Montgomery products of the table (x^2, then the odd powers up to
    x^(2^w - 1)) and of the powering."""
    sched = sliding_schedule(e, w)
    return (1 << (w - 1)) + sum(nsq for nsq, _ in sched[1:]) + sum(1 for _, d in sched[1:] if d)


def montgomery_products_per_encrypt(nbits_n: int, n: int, window: int) -> tuple[int, int]:
    """Montgomery products in the encryption schedule (g^m and r R before,
    the table and sliding-window powering of r^n, one product after) and the
    algorithmic 32x32-bit limb products they stand for (2 S^2 + S with S
    32-bit limbs of n^2, the textbook CIOS count)."""
    mm = 2 + schedule_products(n, window) + 1
    S = 2 * ((nbits_n + 31) // 32)
    return mm, mm * (2 * S * S + S)


def montgomery_products_per_decrypt(p: int, q: int, window: int) -> tuple[int, int]:
    """Both CRT halves: reduction of c + R^3 product + table + sliding-window
    powering of c^(s-1) + conversion."""
    total_mm, total_prod = 0, 0
    for s in (p, q):
        mm = 2 + schedule_products(s - 1, window) + 1
        S = (s * s).bit_length() + 31 >> 5
        total_mm += mm
        total_prod += mm * (2 * S * S + S)
    return total_mm, total_prod


# MI355X i8 matrix cores, dense: 5.0 POP/s = 2.5e15 multiply-accumulates/s
PEAK_I8_MACS = 2.5e15
MFMA_S = {256: 10, 512: 19, 1024: 37, 2048: 74, 4096: 147, 6144: 220, 8192: 293}


def mfma_per_product(nbits_n2: int) -> int:
    """v_mfma_i32_16x16x64_i8 instructions per Montgomery product of the
    matrix-core engine: the tiles of T = x y, of q (the low S limbs) and of
    q N from the tile holding limb S - 2 up, each over the Toeplitz bands
    that reach it."""
    S = MFMA_S[nbits_n2]
    D = 4 * S
    tmin, tmax, umin, umax = -3, (D + 62) // 64, -1, (D - 1) // 64

    def tiles(q0, ntq):
        return sum(1 for q in range(q0, ntq) for t in range(tmin, tmax + 1)
                   if umin <= 4 * q - t <= umax)
    nt, ntlo, qlo = (2 * S + 1 + 63) // 64, (S + 63) // 64, (S - 2) // 64
    return tiles(0, nt) + tiles(0, ntlo) + tiles(qlo, nt)


# the library's automatic window width at 2048 to 4096 bits, for either
# Montgomery engine
AUTO_WINDOW = 6


def roofline_valu(products: float, secs: float) -> dict:
    """VALU engine: algorithmic 32x32-bit limb products per second against
    one v_mad_u64_u32 per lane per clock."""
    a = products / secs
    return {"bound": "alu", "unit": "T limb-products/s (32x32->64, v_mad_u64_u32)",
            "achieved": round(a / 1e12, 3), "peak": round(PEAK_PRODUCTS / 1e12, 3),
            "frac": round(a / PEAK_PRODUCTS, 4)}


def roofline_mfma(nbits_n: int, mm: int, count: int, secs: float) -> dict:
    """i8 matrix-core engine: the algorithmic work of a Montgomery product
    is 2 d^2 multiply-accumulates of bytes (x y and the reduction, d = bytes
    of n^2), two int8 operations each, against the dense int8 peak; issued:
    the 16 x 16 x 64 matrix instructions the engine runs."""
    d = 2 * nbits_n // 8
    ops = 2.0 * count * mm * 2 * d * d / secs
    issued = 2.0 * count * mm * mfma_per_product(2 * nbits_n) * 16 * 16 * 64 / secs
    return {"bound": "mfma", "unit": "TOP/s (int8, 2 per multiply-accumulate)",
            "achieved": round(ops / 1e12, 1), "peak": round(2 * PEAK_I8_MACS / 1e12, 1),
            "frac": round(ops / (2 * PEAK_I8_MACS), 4),
            "issued_frac": round(issued / (2 * PEAK_I8_MACS), 4),
            "mfma_per_product": mfma_per_product(2 * nbits_n)}


# ------------------------------------------------------- measured HBM traffic
# Per kernel: the committed FETCH_SIZE / WRITE_SIZE record and the sources
# that define the kernel; a record counts only while they are unchanged
# since its counters were taken.
TRAFFIC = {
    "k_encrypt": ("k_encrypt_2048bit_traffic.json",
                  ["kernels_paillier.hip", "paillier_ops.hpp", "engine.hpp", "mont_tile.hpp",
                   "bn_scalar.hpp", "pc2_types.hpp", "launch.hpp"]),
    "k_encrypt_mfma": ("k_encrypt_mfma_2048bit_traffic.json",
                       ["kernels_mfma.hip", "mfma_mont.hpp", "paillier_ops.hpp", "pc2_types.hpp",
                        "launch.hpp"]),
}


def kernel_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC[kernel][1]:
        with open(os.path.join(ROOT, "paper_2601_14980_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, elements: int):
    """HBM bytes per launch of `kernel` over `elements` from its committed
    FETCH_SIZE / WRITE_SIZE record, or None if the kernel changed since."""
    try:
        with open(os.path.join(ROOT, "profiles", TRAFFIC[kernel][0])) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_source_hash(kernel) or rec.get("elements") != elements:
        return None
    return int(rec["hbm_bytes_per_launch"])


# ------------------------------------------------------------- CPU baseline
def _oracle_job(args):
    kind, key, a, b = args
    from oracle import paillier as O
    if kind == "enc":
        return O.encrypt(key, a, b)
    return O.decrypt(key, a)


# key sizes of the oracle timing and the seeds of their keys (the workloads'
# own keys: tiny, batching 1024-bit, main 2048-bit, lasso 3072-bit)
CPU_SIZES = ((256, 1), (1024, 3), (2048, 2), (3072, 4))
CPU_ONE_CORE = 8


def cpu_baseline(pc2, gen, ctx, torch, np) -> dict:
    """The oracle as it stands, timed on the host's cores: per key size,
    max(256, 8 cores) encryptions and as many decryptions over every core
    (a process pool), and CPU_ONE_CORE of each in this process alone.  The
    same (m, r) are encrypted and the resulting ciphertexts decrypted by the
    GPU, and every oracle output is compared with the GPU's."""
    from oracle import paillier as O
    from workload.limbs import ints_from_limbs, to_limbs
    cores = len(os.sched_getaffinity(0))
    count = max(256, 8 * cores)
    rows, exact = {}, True
    with mp.get_context("fork").Pool(cores) as pool:
        for bits, seed in CPU_SIZES:
            p, q = gen.primes_for(seed, bits)
            n = p * q
            pk, sk = O.derive_keys(p, q)
            rng = np.random.default_rng(gen.seed_seq(seed, gen.DATA, 77))
            ms = [int(v) for v in rng.integers(0, 1 << 24, size=count)]
            rs = gen.gen_r(n, count, seed, extra=77)
            gsk = pc2.SecretKey(ctx, bits, p, q)
            L = gsk.L
            c_dev = torch.empty((count, 2 * L), dtype=torch.int32, device="cuda")
            m_dev = torch.empty((count, L), dtype=torch.int32, device="cuda")
            pc2.pc2_encrypt(gsk.public, pc2.to_device_limbs(to_limbs(ms, 1)),
                            pc2.to_device_limbs(to_limbs(rs, L)), c_dev)
            pc2.pc2_decrypt(gsk, c_dev, m_dev)
            if ctx.sync() != 0:
                raise RuntimeError("device reported a data error in the oracle sample")
            c_gpu = ints_from_limbs(pc2.from_device_limbs(c_dev))
            m_gpu = ints_from_limbs(pc2.from_device_limbs(m_dev))
            gsk.close()
            t0 = time.perf_counter()
            c_cpu = pool.map(_oracle_job, [("enc", pk, m, r) for m, r in zip(ms, rs)], chunksize=1)
            t1 = time.perf_counter()
            m_cpu = pool.map(_oracle_job, [("dec", sk, c, None) for c in c_gpu], chunksize=1)
            t2 = time.perf_counter()
            k = CPU_ONE_CORE
            for j in range(k):
                c_cpu[j] = O.encrypt(pk, ms[j], rs[j])
            t3 = time.perf_counter()
            for j in range(k):
                m_cpu[j] = O.decrypt(sk, c_gpu[j])
            t4 = time.perf_counter()
            same = c_cpu == c_gpu and m_cpu == m_gpu and m_gpu == ms
            exact &= same
            rows[str(bits)] = {
                "enc_per_s": round(count / (t1 - t0), 2), "dec_per_s": round(count / (t2 - t1), 2),
                "enc_dec_ops_per_s": round(2 * count / (t2 - t0), 2),
                "one_core_enc_per_s": round(k / (t3 - t2), 3),
                "one_core_dec_per_s": round(k / (t4 - t3), 3),
                "equal_to_gpu": same}
            log(f"oracle {bits}-bit: {rows[str(bits)]['enc_dec_ops_per_s']} enc+dec ops/s on "
                f"{cores} cores, one core {rows[str(bits)]['one_core_enc_per_s']} enc/s, "
                f"equal to the GPU: {same}")
    main = rows["2048"]
    return {"value": main["enc_dec_ops_per_s"], "unit": "ops/s", "cores": cores, "kind": "oracle",
            "sample": f"{count} encryptions + {count} decryptions per key size (256, 1024, 2048, "
                      f"3072 bits) over a pool of {cores} processes, {CPU_ONE_CORE} + "
                      f"{CPU_ONE_CORE} on one core; value: the 2048-bit enc+dec rate on all "
                      f"cores; every oracle output compared with the GPU's",
            "cpu_model": _cpu_model(), "by_key_bits": rows, "all_equal_to_gpu": bool(exact)}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


# ------------------------------------------------------- batching (config 3)
BATCH_NODES = 16
BATCH_SEED = 3


def run_batching(pc2, gen, ctx, torch, np, args, reps: int = 3) -> dict:
    """16 nodes, lengths log-uniform in [1024, 65536], even nodes under a
    1024-bit key and odd nodes under a 2048-bit key.  Phases: encrypt every
    node vector; per key group, multiply element j over the nodes whose
    vector reaches j; decrypt both aggregates.  Batched: one persistent
    graph-captured launch per phase.  Plain: one launch per call.  The
    encryption tile (lanes per ciphertext) and the windows of both key
    sizes come from the autotuner first; both paths use them."""
    lengths = gen.log_uniform_lengths(BATCH_SEED, BATCH_NODES, 1024, 65536)
    keys = []
    tuned = {}
    for bits in (1024, 2048):
        p, q = gen.primes_for(BATCH_SEED, bits)
        keys.append(pc2.SecretKey(ctx, bits, p, q))
        t1 = time.perf_counter()
        we, wd, te = pc2.pc2_autotune(keys[-1])
        tuned[str(bits)] = {"enc_lanes": te, "enc_window": we, "dec_window": wd,
                            "tuning_s": round(time.perf_counter() - t1, 2)}
        log(f"autotune {bits}-bit: encryption {te} lanes, w {we}; decryption w {wd}")
    xs = gen.normal_vectors(BATCH_SEED, lengths)
    qp = gen.Q_PLAIN
    nodes = []
    for i, L in enumerate(lengths):
        sk = keys[i % 2]
        x = torch.from_numpy(xs[i]).cuda()
        m = torch.empty(L, dtype=torch.int64, device="cuda")
        pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, qp.delta, x, m)
        r = pc2.to_device_limbs(gen.gen_r_limbs(sk.n, L, sk.L, BATCH_SEED, extra=i))
        c = torch.empty((L, 2 * sk.L), dtype=torch.int32, device="cuda")
        nodes.append(dict(sk=sk, L=L, m=m.view(torch.int32).reshape(L, 2), r=r, c=c))
    groups = []
    for g, sk in enumerate(keys):
        mem = [nd for i, nd in enumerate(nodes) if i % 2 == g]
        maxlen = max(nd["L"] for nd in mem)
        groups.append(dict(sk=sk, mem=mem, maxlen=maxlen,
                           agg=torch.empty((maxlen, 2 * sk.L), dtype=torch.int32, device="cuda"),
                           dec=torch.empty((maxlen, sk.L), dtype=torch.int32, device="cuda")))
    if ctx.sync() != 0:
        raise RuntimeError("quantize reported a range error")
    enc_jobs = [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["sk"].public, m=nd["m"], r=nd["r"],
                     out=nd["c"]) for nd in nodes]
    sum_jobs = [dict(op=pc2.PC2_OP_HOM_SUM, pk=g["sk"].public, inputs=[nd["c"] for nd in g["mem"]],
                     lengths=[nd["L"] for nd in g["mem"]], out=g["agg"]) for g in groups]
    dec_jobs = [dict(op=pc2.PC2_OP_DECRYPT, sk=g["sk"], c=g["agg"], out=g["dec"]) for g in groups]
    batches = [pc2.Batch(ctx, j) for j in (enc_jobs, sum_jobs, dec_jobs)]
    # a HIP stream of default priority made directly: torch.cuda.Stream()
    # would create torch's whole stream pool, after which HIP can map the
    # serving leg's three streams onto shared hardware queues
    hip = ctypes.CDLL("libamdhip64.so")
    side = ctypes.c_void_p()
    if hip.hipStreamCreateWithFlags(ctypes.byref(side), ctypes.c_uint(1)) != 0:
        raise RuntimeError("hipStreamCreateWithFlags failed")

    def batched():
        for b in batches:
            b.run(side.value)
        if hip.hipStreamSynchronize(side) != 0:
            raise RuntimeError("hipStreamSynchronize failed")

    def plain():
        for nd in nodes:
            pc2.pc2_encrypt(nd["sk"].public, nd["m"], nd["r"], nd["c"])
            ctx.sync()
        for g in groups:
            # ragged product as one call per run of equal membership
            cuts = sorted({0} | {nd["L"] for nd in g["mem"]})
            for a, b in zip(cuts[:-1], cuts[1:]):
                ins = [nd["c"][a:b] for nd in g["mem"] if nd["L"] >= b]
                pc2.pc2_hom_sum(g["sk"].public, ins, g["agg"][a:b])
                ctx.sync()
        for g in groups:
            pc2.pc2_decrypt(g["sk"], g["agg"], g["dec"])
            ctx.sync()

    ops = sum(lengths) + sum(g["maxlen"] for g in groups)
    batched()
    plain()
    tb, tp = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        batched()
        tb.append(time.perf_counter() - t1)
        dec_b = [g["dec"].clone() for g in groups]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain()
        tp.append(time.perf_counter() - t1)
        for g, d in zip(groups, dec_b):
            if not torch.equal(g["dec"], d):
                raise RuntimeError("batched and plain results differ")
    if ctx.sync() != 0:
        raise RuntimeError("device reported a data error")
    # exact end-to-end check: decrypted aggregate = sum of quantized plaintexts reaching j
    exact = True
    for g in groups:
        dec = pc2.from_device_limbs(g["dec"])
        want = np.zeros(g["maxlen"], dtype=object)
        for nd in g["mem"]:
            mv = nd["m"].cpu().numpy().view(np.uint64).reshape(-1)
            want[:nd["L"]] += mv.astype(object)
        got = dec[:, 0].astype(object) + (dec[:, 1].astype(object) << 32)
        exact &= bool(np.all(dec[:, 2:] == 0)) and bool(np.all(got == want))
    for b in batches:
        b.close()
    hip.hipStreamDestroy(side)
    mb, mp = float(np.median(tb)), float(np.median(tp))
    log(f"batching: batched {mb * 1e3:.1f} ms, plain {mp * 1e3:.1f} ms per phase set")
    return {"workload": "16 nodes, lengths log-uniform [1024, 65536] (sum %d), keys 1024/2048-bit "
                        "alternating; encrypt all, ragged per-key aggregation, decrypt both"
                        % sum(lengths),
            "ops": ops, "batched_ops_per_s": round(ops / mb, 1),
            "plain_ops_per_s": round(ops / mp, 1), "batched_over_plain": round(mp / mb, 3),
            "batched_ms": round(mb * 1e3, 2), "plain_ms": round(mp * 1e3, 2),
            "autotuned": tuned, "end_to_end_exact": exact}


# -------------------------------------------------------- serving (config 5)
SERVE_SEED = 5
# requests admitted longer ago than this go first under the shortest-first policy
SERVE_MAX_AGE = 1.0


def run_serving(pc2, gen, ctx, sk, torch, np, args) -> dict:
    """Poisson arrivals of encrypt / aggregate / decrypt requests (1/3 each),
    lengths log-uniform in [256, 65536], the 2048-bit key resident, K ~ U{2..8}
    resident ciphertext vectors per aggregate, admission by a 4 GiB budget.

    The plain path serves the configured trace (2000 req/s) one request at a
    time in arrival order, each as one synchronous call (one launch per call,
    no batching or overlap); its outputs are every request's result run
    alone.  libpc2's request server then serves the same trace at 2000 req/s
    (overload: latency is queueing) and at 0.7x the capacity it measured
    there (the same requests, arrivals spread out), and every request's
    output of every served run is compared with its alone result."""
    from paper_2601_14980_amd.serve import Request, percentile, serve_trace
    import random
    L = sk.L
    PL = 65536
    rng = np.random.default_rng(gen.seed_seq(SERVE_SEED, gen.DATA))
    xq = torch.from_numpy(rng.standard_normal(PL)).cuda()
    qp = gen.Q_PLAIN
    mpool = torch.empty(PL, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, qp.delta, xq, mpool)
    mpool2 = mpool.view(torch.int32).reshape(PL, 2)
    rpool = pc2.to_device_limbs(gen.gen_r_limbs(sk.n, PL, L, SERVE_SEED))
    cpool = []
    for k in range(8):
        c = torch.empty((PL, 2 * L), dtype=torch.int32, device="cuda")
        cpool.append(c)
    pc2.pc2_encrypt(sk.public, mpool2, rpool, cpool[0])
    for k in range(1, 8):  # distinct resident ciphertexts: powers of the first
        kk = torch.full((PL,), k + 1, dtype=torch.int64, device="cuda")
        pc2.pc2_hom_scalar_mul(sk.public, cpool[0], kk, cpool[k])
    if ctx.sync() != 0:
        raise RuntimeError("device reported a data error while warming the pool")

    def make_trace(n, rate, seed):
        """n requests; the same seed gives the same requests at any rate
        (only the gaps between arrivals scale)."""
        r = random.Random(seed)
        t, out = 0.0, []
        for i in range(n):
            t += r.expovariate(rate)
            op = ("encrypt", "aggregate", "decrypt")[r.randrange(3)]
            length = int(round(np.exp(r.uniform(np.log(256), np.log(65536)))))
            req = Request(rid=i, op=op, length=length, arrival=t)
            width = L if op == "decrypt" else 2 * L
            res = torch.empty((length, width), dtype=torch.int32, device="cuda")
            if op == "encrypt":
                req.payload = dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=mpool2[:length],
                                   r=rpool[:length], out=res)
            elif op == "aggregate":
                req.K = r.randint(2, 8)
                req.payload = dict(op=pc2.PC2_OP_HOM_SUM, pk=sk.public,
                                   inputs=[cpool[j] for j in r.sample(range(8), req.K)], out=res)
            else:
                req.payload = dict(op=pc2.PC2_OP_DECRYPT, sk=sk,
                                   c=cpool[r.randrange(8)][:length], out=res)
            out.append(req)
        return out

    budget = 4 << 30
    n = args.serve_requests
    enc_dec = lambda reqs: sum(r.length for r in reqs if r.op in ("encrypt", "decrypt"))

    def summary(reqs, span):
        lat = [r.latency for r in reqs]
        return dict(requests=len(reqs),
                    rate_req_per_s=round(len(reqs) / max(reqs[-1].arrival - reqs[0].arrival,
                                                         1e-9), 1),
                    p50_ms=round(1e3 * percentile(lat, 50), 2),
                    p99_ms=round(1e3 * percentile(lat, 99), 2),
                    makespan_s=round(span, 3),
                    enc_dec_ops_per_s=round(enc_dec(reqs) / span, 1),
                    elements_per_s=round(sum(r.length for r in reqs) / span, 1))

    def plain(reqs):
        """One request at a time in arrival order, each one synchronous call."""
        clock = time.perf_counter
        start = clock()
        for r in reqs:
            r.arrival += start
        for r in sorted(reqs, key=lambda q: (q.arrival, q.rid)):
            while clock() < r.arrival:
                time.sleep(min(1e-3, max(0.0, r.arrival - clock())))
            job = r.payload
            if r.op == "encrypt":
                pc2.pc2_encrypt(sk.public, job["m"], job["r"], job["out"])
            elif r.op == "aggregate":
                pc2.pc2_hom_sum(sk.public, [c[:r.length] for c in job["inputs"]], job["out"])
            else:
                pc2.pc2_decrypt(sk, job["c"], job["out"])
            if ctx.sync() != 0:
                raise RuntimeError("device reported a data error on the plain path")
            r.completed = clock()
        return clock() - start

    def serve(reqs, ref, policy):
        srv = pc2.Server(ctx, sk, hbm_budget=budget, tick_groups=args.serve_tick_groups,
                         max_requests=max(1024, 2 * len(reqs)))
        srv.set_policy(policy, SERVE_MAX_AGE)
        span = serve_trace(srv, reqs)
        torch.cuda.synchronize()
        st = srv.stats()
        srv.close()
        if ctx.sync() != 0:
            raise RuntimeError("device reported a data error while serving")
        out = summary(reqs, span)
        out.update(launches=st["launches"], max_hbm_bytes=st["max_bytes"],
                   all_requests_equal_alone=all(torch.equal(a.payload["out"], b.payload["out"])
                                                for a, b in zip(reqs, ref)))
        return out

    ref = make_trace(n, 2000.0, SERVE_SEED)
    plain_run = summary(ref, plain(ref))
    log(f"serving (plain path, {n} requests): p50 {plain_run['p50_ms']} ms p99 "
        f"{plain_run['p99_ms']} ms, {plain_run['enc_dec_ops_per_s']} enc+dec ops/s")
    hot = serve(make_trace(n, 2000.0, SERVE_SEED), ref, pc2.PC2_SERVE_SHORTEST)
    cap = hot["requests"] / hot["makespan_s"]
    sub = serve(make_trace(n, 0.7 * cap, SERVE_SEED), ref, pc2.PC2_SERVE_SHORTEST)
    runs = [("shortest first", hot, sub)]
    out = {"workload": f"{n} requests per run, Poisson arrivals, encrypt/aggregate/decrypt 1/3 "
                       "each, lengths log-uniform [256, 65536], 2048-bit key, HBM budget 4 GiB, "
                       "libpc2 request server; the plain path serves the same trace one "
                       "synchronous call per request",
           "tick_groups": args.serve_tick_groups,
           "policy": f"shortest remaining first, requests older than {SERVE_MAX_AGE} s first",
           "configured_2000_req_s": hot, "sub_saturation_0p7_capacity": sub,
           "plain_path_2000_req_s": plain_run,
           "served_over_plain": round(hot["enc_dec_ops_per_s"] / plain_run["enc_dec_ops_per_s"],
                                      3)}
    if args.serve_fair:
        hot_f = serve(make_trace(n, 2000.0, SERVE_SEED), ref, pc2.PC2_SERVE_FAIR)
        sub_f = serve(make_trace(n, 0.7 * cap, SERVE_SEED), ref, pc2.PC2_SERVE_FAIR)
        runs.append(("fair share", hot_f, sub_f))
        out["fair_share"] = {"configured_2000_req_s": hot_f, "sub_saturation_0p7_capacity": sub_f}
    for name, h, u in runs:
        log(f"serving ({name}): offered 2000 req/s -> p50 {h['p50_ms']} ms p99 {h['p99_ms']} ms; "
            f"at 0.7x capacity ({0.7 * cap:.0f} req/s) p50 {u['p50_ms']} ms p99 {u['p99_ms']} ms; "
            f"every request equal alone: {h['all_requests_equal_alone']} / "
            f"{u['all_requests_equal_alone']}")
    return out


# ------------------------------------------------------------- ADMM (config 4)
ADMM_SEED = 4
ADMM_BITS = 3072
ADMM_M, ADMM_N, ADMM_K = 4096, 16384, 32


# ------------------------------------------- column-split ADMM (Algorithm 1)
COLSPLIT_SEED = 8


def run_colsplit(pc2, gen, ctx, sk, torch, np, args) -> dict:
    """Algorithm 1 with A split by columns, at the paper's shape by default:
    A 3000 x 27000 ~ N(0, 1/M) over 3 nodes of 9000 columns, x* 5 %-sparse
    with N(0,1) nonzeros, noise 1e-3, rho = 1, lambda = 0.1 ||A^T y||_inf,
    the 2048-bit key.  The float64 set-up runs once; the float64 loop without
    quantization runs T iterations; then for each quantization scale 2^k of
    the sweep (Delta = 16 2^k on [-8, 8): k = 13 .. 46 spans Delta = 1e5 ..
    1e15) the object is quantized again and the encrypted loop runs T
    iterations from zero.  Reported per scale: the mean squared and largest
    difference of z from the float64 loop's (the quantization loss the
    paper's Delta sweep measures), the MSE of z against x*, and the time of
    one encrypted iteration (encrypt 2N, hom_add N, K ciphertext mat-vecs of
    N/K x N/K, decrypt N, inverse quantization, update)."""
    from paper_2601_14980_amd.colsplit import ColumnSplitLasso
    M, N, K, T = args.colsplit_m, args.colsplit_n, 3, args.colsplit_iters
    scales = args.colsplit_scales
    rng = np.random.default_rng(gen.seed_seq(COLSPLIT_SEED, gen.DATA))
    A = rng.standard_normal((M, N)) / np.sqrt(M)
    xs = np.zeros(N)
    idx = rng.choice(N, size=N // 20, replace=False)
    xs[idx] = rng.standard_normal(idx.size)
    y = A @ xs + 1e-3 * rng.standard_normal(M)
    lam = 0.1 * float(np.max(np.abs(A.T @ y)))
    Ad, yd = torch.from_numpy(A).cuda(), torch.from_numpy(y).cuda()
    del A
    pool = pc2.to_device_limbs(gen.gen_r_limbs(sk.n, 3 * N, sk.L, COLSPLIT_SEED))
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    cs = ColumnSplitLasso(ctx, sk, Ad, yd, K, 1.0, scales[0], pool)
    setup_s = time.perf_counter() - t0
    log(f"colsplit {M}x{N} over {K} nodes: set-up {setup_s:.1f} s")

    def loop(quantized):
        cs.x.zero_(), cs.z.zero_(), cs.v.zero_()
        ms = []
        for _ in range(T):
            ev[0].record(stream)
            cs.iterate(lam, quantized=quantized)
            ev[1].record(stream)
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        if ctx.sync() != 0:
            raise RuntimeError("device reported a data error in the column-split loop")
        return cs.z.cpu().numpy(), float(np.median(ms))

    zp, plain_ms = loop(False)
    sweep = []
    for i, k in enumerate(scales):
        t1 = time.perf_counter()
        if i:
            cs.set_scale(k)
        rescale_s = time.perf_counter() - t1
        zq, it_ms = loop(True)
        row = {"log2_scale": k, "delta": 16 * 2 ** k,
               "mse_vs_float64": float(np.mean((zq - zp) ** 2)),
               "max_abs_vs_float64": float(np.max(np.abs(zq - zp))),
               "mse_vs_xstar": float(np.mean((zq - xs) ** 2)),
               "iteration_ms": round(it_ms, 2), "quantize_again_s": round(rescale_s, 2)}
        sweep.append(row)
        log(f"colsplit 2^{k}: MSE vs float64 {row['mse_vs_float64']:.3e}, vs x* "
            f"{row['mse_vs_xstar']:.3e}, {row['iteration_ms']:.1f} ms per iteration")
    cs.close()
    return {"workload": f"A {M}x{N} ~ N(0,1/{M}) split by columns over {K} nodes, x* 5% sparse, "
                        f"noise 1e-3, rho 1, lambda {lam:.4g}, 2048-bit key, {T} iterations "
                        f"per scale from zero",
            "setup_s": round(setup_s, 2), "float64_iteration_ms": round(plain_ms, 2),
            "float64_mse_vs_xstar": float(np.mean((zp - xs) ** 2)), "sweep": sweep}


# -------------------------------------------------------- 4096-bit keys
KEY4096_SEED = 7


def run_key4096(pc2, gen, ctx, torch, np, args) -> dict:
    """Encryption and CRT decryption under a 4096-bit key (n^2 of 8192 bits),
    the largest key of the paper's timing table: quantized N(0,1) data, one
    launch per call, then every decryption compared with its plaintext."""
    count = args.key4096_count
    nbits = 4096
    t0 = time.perf_counter()
    p, q = gen.primes_for(KEY4096_SEED, nbits)
    sk = pc2.SecretKey(ctx, nbits, p, q)
    log(f"4096-bit key generated in {time.perf_counter() - t0:.1f}s")
    L = sk.L
    rng = np.random.default_rng(gen.seed_seq(KEY4096_SEED, gen.DATA))
    qp = gen.Q_PLAIN
    x = torch.from_numpy(rng.standard_normal(count)).cuda()
    mq = torch.empty(count, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, qp.delta, x, mq)
    m2 = mq.view(torch.int32).reshape(count, 2)
    r = pc2.to_device_limbs(gen.gen_r_limbs(sk.n, count, L, KEY4096_SEED))
    c = torch.empty((count, 2 * L), dtype=torch.int32, device="cuda")
    d = torch.empty((count, L), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    te, td = [], []
    for rep in range(3):                      # rep 0 warms up
        ev[0].record(stream)
        pc2.pc2_encrypt(sk.public, m2, r, c)
        ev[1].record(stream)
        pc2.pc2_decrypt(sk, c, d)
        ev[2].record(stream)
        torch.cuda.synchronize()
        if rep:
            te.append(ev[0].elapsed_time(ev[1]))
            td.append(ev[1].elapsed_time(ev[2]))
    ok = ctx.sync() == 0
    dh = d.cpu()
    ok &= bool(torch.equal(dh[:, :2], m2.cpu())) and bool((dh[:, 2:] == 0).all())
    # the automatic engine choice runs 4096-bit encryptions on the matrix cores
    engine = ctx.get_option(pc2.PC2_OPT_MODMUL)
    mfma = engine in (pc2.PC2_MODMUL_MFMA, pc2.PC2_MODMUL_AUTO)
    mm_e, prod_e = montgomery_products_per_encrypt(nbits, sk.n, AUTO_WINDOW)
    mm_d, prod_d = montgomery_products_per_decrypt(p, q, AUTO_WINDOW)
    me, md = float(np.median(te)) / 1e3, float(np.median(td)) / 1e3
    roof = (roofline_mfma(nbits, mm_e, count, me) if mfma
            else roofline_valu(prod_e * count, me))
    log(f"4096-bit: encrypt {count} in {me * 1e3:.1f} ms ({'mfma' if mfma else 'valu'} engine), "
        f"decrypt in {md * 1e3:.1f} ms, round trip exact {ok}")
    return {"workload": f"4096-bit key (n^2 8192 bits), {count} quantized N(0,1) values: "
                        "encrypt, then decrypt, one launch per call",
            "encrypt_engine": "mfma" if mfma else "valu",
            "enc_per_s": round(count / me, 1), "dec_per_s": round(count / md, 1),
            "enc_dec_ops_per_s": round(2 * count / (me + md), 1),
            "mm_per_encrypt": mm_e, "mm_per_decrypt": mm_d,
            "encrypt_roofline": roof,
            "round_trip_exact": bool(ok)}


# ------------------------------------------- ciphertext mat-vec (column form)
MATVEC_SEED = 6
MATVEC_EBITS = 50


def run_matvec(pc2, gen, ctx, sk, torch, np, args) -> dict:
    """The edge node's update in the paper's column form: out_i = alpha_i *
    prod_j c_j^(B_ij) mod n^2 under the 2048-bit key, B a dim x dim matrix of
    50-bit constants (the quantized matrix of a node when 27000 columns are
    split over 3 nodes), c and alpha encryptions of quantized N(0,1) data.
    One timed repetition = building the fixed-base tables of c plus applying
    every row.  Checked exactly: the outputs of 64 sampled rows decrypt to
    alpha + B m computed with host integers."""
    D = args.matvec_dim
    L = sk.L
    rng = np.random.default_rng(gen.seed_seq(MATVEC_SEED, gen.DATA))
    qp = gen.Q_PLAIN
    x = torch.from_numpy(rng.standard_normal(2 * D)).cuda()
    mq = torch.empty(2 * D, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, qp.delta, x, mq)
    r = pc2.to_device_limbs(gen.gen_r_limbs(sk.n, 2 * D, L, MATVEC_SEED))
    enc = torch.empty((2 * D, 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_encrypt(sk.public, mq.view(torch.int32).reshape(2 * D, 2), r, enc)
    c, alpha = enc[:D], enc[D:]
    Bh = (rng.integers(0, 1 << 62, size=(D, D), dtype=np.int64, endpoint=False)
          >> (62 - MATVEC_EBITS))
    B = torch.from_numpy(Bh).cuda()
    out = torch.empty((D, 2 * L), dtype=torch.int32, device="cuda")
    if ctx.sync() != 0:
        raise RuntimeError("device reported a data error while preparing the mat-vec")
    mv = pc2.MatVec(sk.public, D, MATVEC_EBITS, 0, rows_hint=D)
    w, nw = mv.window, -(-MATVEC_EBITS // mv.window)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_tab, t_app = [], []
    for rep in range(3):                      # rep 0 warms up
        ev[0].record(stream)
        mv.load(c)
        ev[1].record(stream)
        mv.apply(B, out, alpha)
        ev[2].record(stream)
        torch.cuda.synchronize()
        if rep:
            t_tab.append(ev[0].elapsed_time(ev[1]))
            t_app.append(ev[1].elapsed_time(ev[2]))
        log(f"matvec rep {rep}: tables {ev[0].elapsed_time(ev[1]):.1f} ms, "
            f"rows {ev[1].elapsed_time(ev[2]):.1f} ms")
    if ctx.sync() != 0:
        raise RuntimeError("device reported a data error in the mat-vec")
    mv.close()
    dec = torch.empty((D, L), dtype=torch.int32, device="cuda")
    pc2.pc2_decrypt(sk, out, dec)
    ok = ctx.sync() == 0
    decs = pc2.from_device_limbs(dec)
    mh = mq.cpu().numpy().astype(object)
    m, a = mh[:D], mh[D:]
    n = sk.n
    sample = np.random.default_rng(1).choice(D, size=min(64, D), replace=False)
    for i in sample:
        want = (int(a[i]) + int(np.dot(Bh[i].astype(object), m))) % n
        got = sum(int(decs[i, k]) << (32 * k) for k in range(L))
        ok &= got == want
    per_mm = 2 * (2 * L) ** 2 + 2 * L
    mm_tab = D * sum(w * t + (1 << w) - 1 for t in range(nw))
    mm_app = D * D * nw
    tt, ta = float(np.median(t_tab)) / 1e3, float(np.median(t_app)) / 1e3
    achieved = (mm_tab + mm_app) * per_mm / (tt + ta)
    log(f"matvec {D}x{D}: w {w}, tables {tt * 1e3:.1f} ms, rows {ta * 1e3:.1f} ms, "
        f"{achieved / 1e12:.2f} T products/s, exact {ok}")
    return {"workload": f"2048-bit key, B {D}x{D} of {MATVEC_EBITS}-bit constants, c and alpha "
                        f"encryptions of quantized N(0,1) data: out = alpha * c^B mod n^2",
            "window": w, "table_bytes": int(D * nw * ((1 << w) - 1) * 640),
            "tables_ms": round(tt * 1e3, 2), "rows_ms": round(ta * 1e3, 2),
            "montgomery_products": mm_tab + mm_app,
            "powers_per_s": round(D * D / (tt + ta), 1),
            "achieved_T_products_per_s": round(achieved / 1e12, 3),
            "frac_of_peak": round(achieved / PEAK_PRODUCTS, 4),
            "sampled_rows_exact": bool(ok)}


def run_admm(pc2, gen, ctx, torch, np, args, engines) -> dict:
    """Distributed lasso, A 4096 x 16384 ~ N(0, 1/4096) split row-wise over 32
    nodes, x* 1 %-sparse with N(0,1) nonzeros, noise 1e-3; rho = 1,
    lambda = 0.1 ||A^T y||_inf.  Every iteration quantizes the 32 local
    16384-dim updates, encrypts them under a 3072-bit key, aggregates them
    homomorphically, decrypts and dequantizes the sum and applies the
    consensus update, all on the device.  The loop runs once per engine of
    the encryptions' Montgomery product ("valu", "mfma": i8 matrix cores),
    each from z = u = 0; the iterates must agree exactly across engines."""
    from paper_2601_14980_amd.admm import EncryptedConsensusLasso
    M, N, K = ADMM_M, ADMM_N, ADMM_K
    t0 = time.perf_counter()
    rng = np.random.default_rng(gen.seed_seq(ADMM_SEED, gen.DATA))
    A = rng.standard_normal((M, N)) / 64.0          # N(0, 1/4096)
    support = rng.choice(N, size=N // 100, replace=False)
    xstar = np.zeros(N)
    xstar[support] = rng.standard_normal(support.size)
    y = A @ xstar + 1e-3 * rng.standard_normal(M)
    lam = 0.1 * float(np.max(np.abs(A.T @ y)))
    p, q = gen.primes_for(ADMM_SEED, ADMM_BITS)
    sk = pc2.SecretKey(ctx, ADMM_BITS, p, q)
    r_pool = pc2.to_device_limbs(gen.gen_r_limbs(p * q, K * N, sk.L, ADMM_SEED))
    log(f"admm: inputs generated in {time.perf_counter() - t0:.1f}s")
    qa = gen.Q_ADMM
    Ad = torch.from_numpy(A).cuda()
    yd = torch.from_numpy(y).cuda()
    del A
    drv = EncryptedConsensusLasso(ctx, sk, Ad, yd, K, 1.0, lam, qa.log2_scale, qa.offset,
                                  qa.delta, r_pool)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    out = {"workload": "lasso A 4096x16384 ~ N(0,1/4096), 32 nodes x 128 rows, x* 1% sparse, "
                       "noise 1e-3, rho 1, lambda 0.1 ||A^T y||_inf; 3072-bit key, scale 2^44, "
                       "offset 2^51", "lambda": lam}
    final = {}
    for engine in engines:
        ctx.set_option(pc2.PC2_OPT_MODMUL,
                       pc2.PC2_MODMUL_MFMA if engine == "mfma" else pc2.PC2_MODMUL_VALU)
        z = torch.zeros(N, dtype=torch.float64, device="cuda")
        u = torch.zeros((K, N), dtype=torch.float64, device="cuda")
        times, enc_ms, dec_ms = [], [], []
        for it in range(args.admm_warmup + args.admm_iters):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            drv.local(z, u)
            pc2.pc2_quantize(ctx, qa.log2_scale, qa.offset, qa.delta, drv.xu.reshape(-1), drv.m)
            ev[0].record(stream)
            pc2.pc2_encrypt(sk.public, drv.m.view(torch.int32).reshape(K * N, 2), drv.r, drv.c)
            ev[1].record(stream)
            pc2.pc2_hom_sum(sk.public, drv.parts, drv.agg)
            ev[2].record(stream)
            pc2.pc2_decrypt(sk, drv.agg, drv.msum)
            ev[3].record(stream)
            pc2.pc2_dequantize(ctx, qa.log2_scale, qa.offset, drv.msum, K, drv.total)
            drv.consensus(z, u)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            if it >= args.admm_warmup:
                times.append(dt)
                enc_ms.append(ev[0].elapsed_time(ev[1]))
                dec_ms.append(ev[2].elapsed_time(ev[3]))
            log(f"admm ({engine}) iteration {it + 1}: {dt * 1e3:.0f} ms")
        ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)
        if ctx.sync() != 0:
            raise RuntimeError("device reported a data error in the ADMM loop")
        zh = z.cpu().numpy()
        final[engine] = zh
        mt = float(np.median(times))
        enc_s = float(np.median(enc_ms)) / 1e3
        mm, prod = montgomery_products_per_encrypt(ADMM_BITS, p * q, AUTO_WINDOW)
        roof = (roofline_mfma(ADMM_BITS, mm, K * N, enc_s) if engine == "mfma"
                else roofline_valu(K * N * prod, enc_s))
        roof["mm_per_encrypt"] = mm
        out[engine] = {"iterations_timed": len(times), "ms_per_iteration": round(mt * 1e3, 1),
                       "encrypt_roofline": roof,
                       "encrypt_ms": round(float(np.median(enc_ms)), 1),
                       "decrypt_ms": round(float(np.median(dec_ms)), 1),
                       "enc_dec_ops_per_s": round((K * N + N) / mt, 1),
                       "mse_z_vs_xstar": float(np.mean((zh - xstar) ** 2)),
                       "nnz_z": int(np.count_nonzero(zh))}
    if len(final) > 1:
        vals = list(final.values())
        out["engines_agree_exactly"] = all(np.array_equal(vals[0], v) for v in vals[1:])

    # Accuracy over a long run: the encrypted aggregate Dec(prod_k Enc(m_k))
    # equals the integer sum of the quantized m_k (no wrap mod n), so the
    # encrypted loop's iterates are those of the loop that sums the quantized
    # values exactly (checked against the encrypted run above after the same
    # number of iterations); it runs T iterations beside the float64 loop
    # without quantization.  The integer sum over the nodes is torch's (int64,
    # exact); every other step is the library's.
    T, t_check = args.admm_mse_iters, args.admm_warmup + args.admm_iters
    runs, snap = {}, None
    for quantized in (True, False):
        z = torch.zeros(N, dtype=torch.float64, device="cuda")
        u = torch.zeros((K, N), dtype=torch.float64, device="cuda")
        for it in range(T):
            drv.local(z, u)
            if quantized:
                pc2.pc2_quantize(ctx, qa.log2_scale, qa.offset, qa.delta, drv.xu.reshape(-1),
                                 drv.m)
                msum = drv.m.view(K, N).sum(dim=0)
                pc2.pc2_dequantize(ctx, qa.log2_scale, qa.offset,
                                   msum.view(torch.int32).reshape(N, 2), K, drv.total)
            else:
                torch.sum(drv.xu, dim=0, out=drv.total)
            drv.consensus(z, u)
            if quantized and it + 1 == t_check:
                snap = z.cpu().numpy()
        if ctx.sync() != 0:
            raise RuntimeError("device reported a data error in the plaintext lasso loops")
        runs[quantized] = z.cpu().numpy()
    drv.close()
    zq, zf = runs[True], runs[False]
    out["long_run"] = {
        "iterations": T,
        "mse_quantized_vs_float64": float(np.mean((zq - zf) ** 2)),
        "max_abs_quantized_vs_float64": float(np.max(np.abs(zq - zf))),
        "mse_z_vs_xstar_quantized": float(np.mean((zq - xstar) ** 2)),
        "mse_z_vs_xstar_float64": float(np.mean((zf - xstar) ** 2)),
        "nnz_z": int(np.count_nonzero(zq)),
        "quantized_loop_equals_encrypted": bool(snap is not None and len(final) > 0
                                                and all(np.array_equal(snap, v)
                                                        for v in final.values())),
    }
    log(f"admm long run ({T} iterations): MSE quantized vs float64 "
        f"{out['long_run']['mse_quantized_vs_float64']:.3e}, vs x* "
        f"{out['long_run']['mse_z_vs_xstar_quantized']:.3e} (float64 "
        f"{out['long_run']['mse_z_vs_xstar_float64']:.3e}); quantized loop equals the encrypted "
        f"one: {out['long_run']['quantized_loop_equals_encrypted']}")
    return out


# --------------------------------------------------------------------- main
def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-fair", action="store_true",
                    help="also serve both loads under the fair-share policy")
    ap.add_argument("--serve-tick-groups", type=int, default=2048,
                    help="element groups per serving launch (16 encryptions each at 2048 bits)")
    ap.add_argument("--no-admm", action="store_true")
    ap.add_argument("--no-matvec", action="store_true")
    ap.add_argument("--no-key4096", action="store_true")
    ap.add_argument("--no-colsplit", action="store_true")
    ap.add_argument("--colsplit-m", type=int, default=3000)
    ap.add_argument("--colsplit-n", type=int, default=27000)
    ap.add_argument("--colsplit-iters", type=int, default=5)
    ap.add_argument("--colsplit-scales", type=int, nargs="+", default=[13, 23, 33, 46])
    ap.add_argument("--key4096-count", type=int, default=32768)
    ap.add_argument("--matvec-dim", type=int, default=9000)
    ap.add_argument("--admm-iters", type=int, default=2)
    ap.add_argument("--admm-warmup", type=int, default=1)
    ap.add_argument("--admm-mse-iters", type=int, default=200,
                    help="iterations of the lasso accuracy run (plaintext-equivalent loops)")
    ap.add_argument("--admm-modmul", default="valu,mfma",
                    help="Montgomery engines to run the lasso leg with (comma-separated)")
    ap.add_argument("--modmul", choices=("auto", "valu", "mfma"), default="auto",
                    help="Montgomery engine of the main leg's encryptions (auto: VALU at 2048 bits)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run an elementwise kernel that reads and writes MIB MiB "
                         "(reference for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs the hot path on a single MI355X "
              "and has no multi-GPU path; use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):          # an elementwise kernel: reads and writes MIB MiB each
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.calibrate_copy, "launches": 3}), flush=True)
        return 0

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
    if args.modmul != "auto":
        ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_MFMA if args.modmul == "mfma"
                       else pc2.PC2_MODMUL_VALU)
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
    sum_ms: list[float] = []
    dec_ms: list[float] = []

    def step_batched(record: bool) -> None:
        pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, qp.delta, x_all, m_all)
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
            sum_ms.append(ev[1].elapsed_time(ev[2]))
            dec_ms.append(ev[2].elapsed_time(ev[3]))

    def step_plain() -> None:
        for k in range(NODES):
            sl = slice(k * LENGTH, (k + 1) * LENGTH)
            pc2.pc2_quantize(ctx, qp.log2_scale, qp.offset, qp.delta, x_all[sl], m_all[sl])
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

    # key-holder encryption (CRT through p^2, q^2) of the same inputs, checked
    # against the public-key ciphertexts of the last timed step
    c_sk = torch.empty_like(c_all)
    ev[0].record(stream)
    pc2.pc2_encrypt_sk(sk, m2_all, r_all, c_sk)
    ev[1].record(stream)
    torch.cuda.synchronize()
    enc_sk_ms = ev[0].elapsed_time(ev[1])
    enc_sk_same = bool(torch.equal(c_sk, c_all)) and ctx.sync() == 0
    del c_sk
    log(f"key-holder encryption: {enc_sk_ms:.1f} ms, identical ciphertexts: {enc_sk_same}")

    # the other Montgomery engine on the same inputs (one launch), for its own
    # roofline; its ciphertexts must be the same
    main_engine = "mfma" if args.modmul in ("auto", "mfma") else "valu"
    other_engine = "valu" if main_engine == "mfma" else "mfma"
    ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_VALU if other_engine == "valu"
                   else pc2.PC2_MODMUL_MFMA)
    c_other = torch.empty_like(c_all)
    ev[0].record(stream)
    pc2.pc2_encrypt(pk, m2_all, r_all, c_other)
    ev[1].record(stream)
    torch.cuda.synchronize()
    other_ms = ev[0].elapsed_time(ev[1])
    other_same = bool(torch.equal(c_other, c_all)) and ctx.sync() == 0
    del c_other
    ctx.set_option(pc2.PC2_OPT_MODMUL, {"auto": pc2.PC2_MODMUL_AUTO, "mfma": pc2.PC2_MODMUL_MFMA,
                                        "valu": pc2.PC2_MODMUL_VALU}[args.modmul])
    log(f"{other_engine} engine: encrypt {other_ms:.1f} ms, identical ciphertexts: {other_same}")

    # the fused path (Dec(prod_k Enc(m_k, r_k)) in one call, the ciphertexts
    # never written out) on the same inputs, against the three calls of a step
    m_nodes = [m2_all[k * LENGTH:(k + 1) * LENGTH] for k in range(NODES)]
    r_nodes = [r_all[k * LENGTH:(k + 1) * LENGTH] for k in range(NODES)]
    fused_out = torch.empty_like(msum)
    fused_ms = []
    for rep in range(2):                      # rep 0 warms up
        ev[0].record(stream)
        pc2.pc2_enc_sum_dec(sk, m_nodes, r_nodes, fused_out)
        ev[1].record(stream)
        torch.cuda.synchronize()
        if rep:
            fused_ms.append(ev[0].elapsed_time(ev[1]))
    fused_same = bool(torch.equal(fused_out, msum)) and ctx.sync() == 0
    unfused_ms = (sum(enc_ms) + sum(sum_ms) + sum(dec_ms)) / len(enc_ms)
    del fused_out
    log(f"fused enc->sum->dec: {fused_ms[0]:.1f} ms vs {unfused_ms:.1f} ms unfused, "
        f"identical: {fused_same}")

    # plain path
    t_plain = []
    for i in range(args.plain_steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step_plain()
        t_plain.append(time.perf_counter() - t1)
        log(f"plain step {i + 1}/{args.plain_steps}: {t_plain[-1] * 1e3:.0f} ms")
    plain_value = ops_per_step / (sum(t_plain) / len(t_plain)) if t_plain else None

    w = ctx.get_option(pc2.PC2_OPT_WINDOW) or AUTO_WINDOW
    mm_enc, prod_enc = montgomery_products_per_encrypt(NBITS, n, w)
    enc_avg_s = sum(enc_ms) / len(enc_ms) / 1e3

    def engine_roofline(engine, secs):
        if engine == "mfma":
            r = {"kernel": f"k_encrypt_mfma<{MFMA_S[2 * NBITS]}>",
                 **roofline_mfma(NBITS, mm_enc, total, secs),
                 "traffic": measured_traffic("k_encrypt_mfma", total),
                 "per_launch_macs": total * mm_enc * 2 * (NBITS // 4) ** 2}
        else:
            r = {"kernel": "k_encrypt", **roofline_valu(prod_enc * total, secs),
                 "traffic": measured_traffic("k_encrypt", total),
                 "per_launch_products": prod_enc * total}
        r.update({"mm_per_encrypt": mm_enc, "avg_launch_ms": round(secs * 1e3, 3)})
        return r

    roofline = engine_roofline(main_engine, enc_avg_s)
    engines = {main_engine: {"encrypt_ms": round(enc_avg_s * 1e3, 2), "roofline": roofline},
               other_engine: {"encrypt_ms": round(other_ms, 2),
                              "roofline": engine_roofline(other_engine, other_ms / 1e3),
                              "identical_ciphertexts": other_same}}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores")
        cpu = cpu_baseline(pc2, gen, ctx, torch, np)

    batching = None if args.no_batching else run_batching(pc2, gen, ctx, torch, np, args)
    serving = None if args.no_serving else run_serving(pc2, gen, ctx, sk, torch, np, args)
    matvec = None if args.no_matvec else run_matvec(pc2, gen, ctx, sk, torch, np, args)
    colsplit = None if args.no_colsplit else run_colsplit(pc2, gen, ctx, sk, torch, np, args)
    key4096 = None if args.no_key4096 else run_key4096(pc2, gen, ctx, torch, np, args)
    admm = None if args.no_admm else run_admm(pc2, gen, ctx, torch, np, args,
                                              args.admm_modmul.split(","))

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
        # encryption (most of a step) multiplies 7-bit digits as i8 on the
        # matrix cores with i32 accumulation, or 32-bit limbs on the VALU;
        # decryption always runs on 32-bit limbs
        "dtype": "i8" if main_engine == "mfma" else "u32",
        "dtypes": {"encrypt": "i8 x i8 -> i32" if main_engine == "mfma" else "u32 x u32 -> u64",
                   "decrypt": "u32 x u32 -> u64"},
        "data": "synthetic",
        "config": {"workload": "2048-bit key, 8 nodes x 65536 float64 ~ N(0,1), scale 2^20, "
                               "offset 2^23: quantize, encrypt 524288, 8-way sum, decrypt 65536, "
                               "dequantize", "nbits": NBITS, "nodes": NODES, "length": LENGTH,
                   "window": w, "path": "batched", "modmul": args.modmul,
                   "encrypt_engine": main_engine},
        "enc_per_s": round(total / enc_avg_s, 1),
        "dec_per_s": round(LENGTH / (sum(dec_ms) / len(dec_ms) / 1e3), 1),
        "key_holder_enc_per_s": round(total / (enc_sk_ms / 1e3), 1),
        "key_holder_enc_identical": enc_sk_same,
        "fused": {"enc_sum_dec_ms": round(fused_ms[0], 2), "unfused_ms": round(unfused_ms, 2),
                  "fused_over_unfused": round(unfused_ms / fused_ms[0], 3),
                  "identical": fused_same,
                  "unfused": "encrypt 524288 + 8-way hom_sum + decrypt 65536 (per-call event "
                             "times of the timed steps)"},
        "plain": ({"value": round(plain_value, 1), "unit": "ops/s",
                   "ms_per_step": round(1e3 * sum(t_plain) / len(t_plain), 2)}
                  if t_plain else None),
        "batched_over_plain": round(value / plain_value, 3) if t_plain else None,
        "end_to_end_exact": exact,
        "roofline": roofline,
        "engines": engines,
        "cpu_baseline": cpu,
        "batching": batching,
        "serving": serving,
        "matvec": matvec,
        "colsplit": colsplit,
        "key4096": key4096,
        "admm": admm,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0 if exact and other_same else 1


if __name__ == "__main__":
    sys.exit(main())
