"""The encrypted consensus-lasso iteration on the GPU against the float64
oracle (GPU test): every iterate within 1e-12 relative, and the decrypted
aggregate equal to the exact sum of the quantized node vectors."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle.admm import ConsensusLasso, quantize_exact
from workload import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,N,K,iters", [(256, 1024, 8, 6), (4096, 16384, 32, 3)],
                         ids=["small", "full_shape"])
def test_encrypted_admm_matches_oracle(gpu_ctx, M, N, K, iters):
    """The full shape is the lasso workload's (A 4096 x 16384 over 32 nodes);
    a 256-bit key keeps the crypto short, the FP64 part is the real size."""
    from paper_2601_14980_amd import pc2
    from paper_2601_14980_amd.admm import EncryptedConsensusLasso

    rng = np.random.default_rng(gen.seed_seq(4, gen.DATA, M))
    A = rng.standard_normal((M, N)) / np.sqrt(M)
    xs = np.where(rng.random(N) < 0.01, rng.standard_normal(N), 0.0)
    y = A @ xs + 1e-3 * rng.standard_normal(M)
    rho = 1.0
    lam = 0.1 * float(np.max(np.abs(A.T @ y)))
    k, o, dl = gen.Q_ADMM.log2_scale, gen.Q_ADMM.offset, gen.Q_ADMM.delta
    p, q = gen.primes_for(4, 256)
    sk = pc2.SecretKey(gpu_ctx, 256, p, q)
    r_pool = pc2.to_device_limbs(gen.gen_r_limbs(p * q, K * N, sk.L, 4))
    drv = EncryptedConsensusLasso(gpu_ctx, sk, torch.from_numpy(A).cuda(),
                                  torch.from_numpy(y).cuda(), K, rho, lam, k, o, dl, r_pool)
    ora = ConsensusLasso(A, y, K, rho, lam)
    z = torch.zeros(N, dtype=torch.float64, device="cuda")
    u = torch.zeros((K, N), dtype=torch.float64, device="cuda")
    zo, uo = np.zeros(N), np.zeros((K, N))
    for it in range(iters):
        drv.local(z, u)
        drv.aggregate()
        assert gpu_ctx.sync() == 0
        xg = drv.x.cpu().numpy()
        xug = drv.xu.cpu().numpy()
        # the decrypted aggregate is the exact integer sum of the quantized vectors
        msum = pc2.from_device_limbs(drv.msum)
        got = msum[:, 0].astype(object) + (msum[:, 1].astype(object) << 32)
        want = sum(quantize_exact(xug[i], k, o).astype(object) for i in range(K))
        assert np.all(msum[:, 2:] == 0) and np.all(got == want), f"iteration {it}"
        drv.consensus(z, u)
        xo, zo, uo, _ = ora.step(zo, uo, (k, o))
        zg, ug = z.cpu().numpy(), u.cpu().numpy()
        for name, g, w in (("x", xg, xo), ("z", zg, zo), ("u", ug, uo)):
            rel = np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-300)
            assert rel <= 1e-12, f"iteration {it}: {name} relative error {rel:.2e}"
    assert np.linalg.norm(zo) > 0  # the threshold did not zero everything
    drv.close()
