"""Plain, slow CPU oracle for the batched Paillier hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or execute anything in this
package.  The product library never calls it, and it shares no code, tables or
constants with the HIP path: it re-derives every key constant from (p, q) and
computes each operation from its textbook definition with Python integers
(crypto) or numpy float64 (the ADMM driver), so that a reader can check it
against the paper line by line.

Modules
-------
paillier  Key derivation, encryption, decryption and the two homomorphic
          operations, written as the plain definitions of Sec. III-B/III-C
          (no Montgomery form, no windows, no CRT on the parity path).
quant     The affine form of the quantizer of Sec. III-A and its inverse.
admm      The consensus-lasso iteration used by the ADMM driver, in float64.
colsplit  The column-split iteration of Algorithm 1 with its quantized,
          homomorphic node step evaluated by the exact plaintext equivalent.
"""
