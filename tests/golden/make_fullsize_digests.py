"""Write `fullsize_<config>.json` beside this file: SHA-256 digests of the
oracle's Paillier ciphertexts (encryption with g = n + 1, Section III-B)
for a regular sample of a full-size workload (the quantized N(0,1) vectors
and the r values of the seeded generators), in chunks of 4096 sampled
elements, and of the element-wise products over the nodes of the sampled
ciphertexts (Definition 1 applied nodes - 1 times; the sample holds every
node's element at each sampled position, since the stride divides the
vector length):

* 2048bit_8x65536 (default): every eighth element of 8 nodes x 65536 under
  the 2048-bit key of seed 2;
* 3072bit_32x16384: every 32nd element of 32 nodes x 16384 (one lasso
  iteration's encryptions) under the 3072-bit key of seed 4;
* 4096bit_1x32768: every eighth element of one launch of 32768 under the
  4096-bit key of seed 7;
* batch_16nodes (`--config batch_16nodes`): the batching workload, 16 nodes
  of log-uniform lengths in [1024, 65536] (seed 3) under a 1024-bit key
  (even nodes) and a 2048-bit key (odd nodes): every eighth element of
  each node, one digest per node, and the ragged products over each key's
  nodes (position j multiplies the nodes longer than j) at the sampled
  positions, one digest per key.

Only `oracle/` computes (quantize, encrypt); `workload/` supplies the seeded
inputs.  The GPU test in `tests/test_gpu_fullsize.py` encrypts the whole
workload in one launch and compares the digests of the same elements, so
every sampled ciphertext is checked bit for bit, at every position of the
launch.

    python tests/golden/make_fullsize_digests.py [--config NAME] [--workers N]

takes 10-20 minutes per configuration on 8 cores (one oracle encryption,
pure-Python square-and-multiply, is ~0.15 s at 2048 bits, ~0.5 s at 3072
and ~1 s at 4096).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import sys
import time
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent.parent
sys.path.insert(0, str(ROOT))

from oracle import paillier as O  # noqa: E402
from oracle import quant as Q  # noqa: E402
from workload import gen  # noqa: E402
from workload.limbs import ints_from_limbs  # noqa: E402

CONFIGS = {  # name: (key bits, nodes, length, key seed, sample stride)
    "2048bit_8x65536": (2048, 8, 65536, 2, 8),
    "3072bit_32x16384": (3072, 32, 16384, 4, 32),
    "4096bit_1x32768": (4096, 1, 32768, 7, 8),
}
DEFAULT = "2048bit_8x65536"
CHUNK = 4096
BATCH = "batch_16nodes"  # seed, nodes, length range, keys (node i: KEY_BITS[i % 2]), stride
B_SEED, B_NODES, B_LO, B_HI, B_KEY_BITS, B_STRIDE = 3, 16, 1024, 65536, (1024, 2048), 8

_opk = None
_nb = 0


def _init(p: int, q: int, nb: int) -> None:
    global _opk, _nb
    _opk, _ = O.derive_keys(p, q)
    _nb = nb


def _encrypt_chunk(pairs: list[tuple[int, int]]) -> bytes:
    return b"".join(O.encrypt(_opk, m, r).to_bytes(_nb, "little") for m, r in pairs)


def batch_main(workers: int) -> int:
    t0 = time.time()
    qp = gen.Q_PLAIN
    lengths = gen.log_uniform_lengths(B_SEED, B_NODES, B_LO, B_HI)
    keys = [(bits, *gen.primes_for(B_SEED, bits)) for bits in B_KEY_BITS]
    xs = gen.normal_vectors(B_SEED, lengths)
    cts: list[list[int]] = [[] for _ in lengths]  # sampled ciphertexts per node
    for g, (bits, p, q) in enumerate(keys):
        n, nb = p * q, 2 * bits // 8
        members = [i for i in range(B_NODES) if i % 2 == g]
        for i in members:
            rk = ints_from_limbs(gen.gen_r_limbs(n, lengths[i], bits // 32, B_SEED, extra=i))
            pairs = [(Q.quantize(float(xs[i][j]), qp.log2_scale, qp.offset, qp.delta), int(rk[j]))
                     for j in range(0, lengths[i], B_STRIDE)]
            work = [pairs[a:a + 256] for a in range(0, len(pairs), 256)]
            with mp.Pool(workers, initializer=_init, initargs=(p, q, nb)) as pool:
                blob = b"".join(pool.imap(_encrypt_chunk, work))
            cts[i] = [int.from_bytes(blob[a * nb:(a + 1) * nb], "little") for a in range(len(pairs))]
            print(f"node {i} ({bits}-bit, {len(pairs)} samples) done, {time.time() - t0:.0f} s",
                  flush=True)
    node_digests = []
    for i, c in enumerate(cts):
        nb = 2 * B_KEY_BITS[i % 2] // 8
        node_digests.append(hashlib.sha256(b"".join(v.to_bytes(nb, "little") for v in c))
                            .hexdigest())
    agg_digests = []
    for g, (bits, p, q) in enumerate(keys):
        opk, _ = O.derive_keys(p, q)
        nb = 2 * bits // 8
        members = [i for i in range(B_NODES) if i % 2 == g]
        mx = max(lengths[i] for i in members)
        agg = b"".join(O.hom_sum(opk, [cts[i][j // B_STRIDE] for i in members if j < lengths[i]])
                       .to_bytes(nb, "little") for j in range(0, mx, B_STRIDE))
        agg_digests.append(hashlib.sha256(agg).hexdigest())
    doc = {
        "what": "SHA-256 per node of the oracle's ciphertexts (little-endian, 2 * key bits / 8 "
                f"bytes each, in element order) of elements 0, {B_STRIDE}, {2 * B_STRIDE}, ... "
                "of each node's vector; and per key of the ragged products over its nodes "
                f"(position j: the nodes longer than j) at positions 0, {B_STRIDE}, ... below "
                "its longest node",
        "definition": "Paillier encryption with g = n + 1 (Section III-B): "
                      "c = g^m r^n mod n^2, m = the quantized value (Section III-A); "
                      "aggregation: Definition 1",
        "workload": {"seed": B_SEED, "nodes": B_NODES, "lengths": lengths,
                     "key_bits": list(B_KEY_BITS), "node_key": "key_bits[node % 2]",
                     "x": f"gen.normal_vectors({B_SEED}, lengths)",
                     "r": f"gen.gen_r_limbs(n, length, key_bits // 32, {B_SEED}, extra=node)",
                     "quantizer": {"log2_scale": qp.log2_scale, "offset": qp.offset,
                                   "delta": qp.delta}},
        "stride": B_STRIDE,
        "node_digests": node_digests,
        "agg_digests": agg_digests,
        "written_by": f"python tests/golden/make_fullsize_digests.py --config {BATCH} "
                      "(oracle/ only)",
    }
    out = HERE / f"fullsize_{BATCH}.json"
    out.write_text(json.dumps(doc, indent=1) + "\n")
    print(f"wrote {out} in {time.time() - t0:.0f} s", flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--config", choices=sorted(CONFIGS) + [BATCH], default=DEFAULT)
    ap.add_argument("--workers", type=int, default=mp.cpu_count())
    args = ap.parse_args()
    if args.config == BATCH:
        return batch_main(args.workers)
    NBITS, NODES, LENGTH, SEED, STRIDE = CONFIGS[args.config]
    out = HERE / f"fullsize_{args.config}.json"
    nb = 2 * NBITS // 8
    t0 = time.time()
    p, q = gen.primes_for(SEED, NBITS)
    n = p * q
    nl = NBITS // 32
    qp = gen.Q_PLAIN
    xs = gen.normal_vectors(SEED, [LENGTH] * NODES)
    elems = list(range(0, NODES * LENGTH, STRIDE))
    pairs = []
    for k in range(NODES):
        rk = ints_from_limbs(gen.gen_r_limbs(n, LENGTH, nl, SEED, extra=k))
        for j in range(0, LENGTH, STRIDE):
            assert (k * LENGTH + j) % STRIDE == 0
            m = Q.quantize(float(xs[k][j]), qp.log2_scale, qp.offset, qp.delta)
            pairs.append((m, int(rk[j])))
    assert len(pairs) == len(elems) and len(pairs) % CHUNK == 0
    chunks = [pairs[i:i + CHUNK] for i in range(0, len(pairs), CHUNK)]
    # the workers take sub-chunks so that progress shows and the load evens out
    sub = 256
    work = [c[i:i + sub] for c in chunks for i in range(0, len(c), sub)]
    parts: list[bytes] = []
    with mp.Pool(args.workers, initializer=_init, initargs=(p, q, nb)) as pool:
        for i, b in enumerate(pool.imap(_encrypt_chunk, work)):
            parts.append(b)
            if (i + 1) % 16 == 0:
                print(f"{(i + 1) * sub} / {len(pairs)} encryptions, {time.time() - t0:.0f} s",
                      flush=True)
    blob = b"".join(parts)
    digests = [hashlib.sha256(blob[i * CHUNK * nb:(i + 1) * CHUNK * nb]).hexdigest()
               for i in range(len(chunks))]
    # aggregates at the sampled positions j = 0, STRIDE, ... of a node's vector
    opk, _ = O.derive_keys(p, q)
    per_node = LENGTH // STRIDE
    cts = [int.from_bytes(blob[i * nb:(i + 1) * nb], "little") for i in range(len(pairs))]
    agg_digests, agg_chunk = [], min(CHUNK, per_node)
    if NODES > 1:
        agg = b"".join(O.hom_sum(opk, [cts[k * per_node + t] for k in range(NODES)])
                       .to_bytes(nb, "little") for t in range(per_node))
        agg_digests = [hashlib.sha256(agg[i * agg_chunk * nb:(i + 1) * agg_chunk * nb]).hexdigest()
                       for i in range(per_node // agg_chunk)]
    doc = {
        "what": f"SHA-256 of the oracle's ciphertexts (little-endian, {nb} bytes each, in element "
                f"order) of elements 0, {STRIDE}, {2 * STRIDE}, ... of the {NBITS}-bit {NODES} x "
                f"{LENGTH} workload, in chunks of {CHUNK} sampled elements",
        "definition": "Paillier encryption with g = n + 1 (Section III-B): "
                      "c = g^m r^n mod n^2, m = the quantized value (Section III-A)",
        "workload": {"nbits": NBITS, "nodes": NODES, "length": LENGTH, "key_seed": SEED,
                     "x": f"gen.normal_vectors({SEED}, [{LENGTH}] * {NODES})",
                     "r": f"gen.gen_r_limbs(n, {LENGTH}, {nl}, {SEED}, extra=node)",
                     "quantizer": {"log2_scale": qp.log2_scale, "offset": qp.offset,
                                   "delta": qp.delta}},
        "stride": STRIDE,
        "chunk": CHUNK,
        "samples": len(pairs),
        "digests": digests,
        "agg_what": f"SHA-256 of prod over the {NODES} nodes of the oracle's ciphertexts mod n^2 "
                    f"at positions 0, {STRIDE}, ... of a node's vector, in chunks of {agg_chunk}",
        "agg_chunk": agg_chunk,
        "agg_digests": agg_digests,
        "written_by": "python tests/golden/make_fullsize_digests.py"
                      + ("" if args.config == DEFAULT else f" --config {args.config}")
                      + " (oracle/ only)",
    }
    out.write_text(json.dumps(doc, indent=1) + "\n")
    print(f"wrote {out} ({len(digests)} digests) in {time.time() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
