"""GPU parity at the full plain and SeBVer/Distill sizes against the oracle's
own results over the whole batch, through the C ABI.

The batch is 2^20 entries of 256-byte messages (synthlog seed 2), n2 = 256,
n1 = 4096, signed by the oracle (tests/oracle_fullsize.py computes the
oracle's results on the host cores in umbrella-sized chunks).  Compared:

* AVer's accept bit and e mod q on the honest batch and on the batch with
  1% of entries carrying one flipped bit of m_t || sigma_t (synthlog
  corruption plan, seed 3), both instantiations;
* every entry's e_t mod q and x_t from the emit form of the AVer hot kernel
  (same variant, same grid, same code as the timed launch), all 2^20;
* Distill of the corrupted batch into 64 umbrellas: the sorted invalid set
  (the oracle verifies every corrupted entry individually, plus a sample of
  the others), CCD^v and all 64 umbrella tags (the oracle's Agg over each
  umbrella's valid signatures), and SeBVer V/U/I;
* the same batch signed under POSLO-C (one signature per epoch, the 4,096
  epoch commitments in the public key): AVer of the honest and of the
  corrupted batch (1% of epochs with one flipped bit of their messages or
  signature), Distill's invalid epochs, CCD^v and umbrella tags, SeBVer
  V/U/I, all against the oracle's POSLO-C over the whole batch.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N, L, LOG2_N1, LOG2_N2, KEY_FIRST, MSG_SEED, N_U, FLIP_SEED = 1 << 20, 256, 12, 8, 0x20, 2, 64, 3
K_FLIPS = N // 100


@pytest.fixture(scope="module")
def gpu(P):
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ctx = P.poslo_ctx_create(0)
    yield torch, ctx
    ctx.close()


def case_for(inst):
    import oracle_fullsize as F
    print(f"oracle over the full batch, inst {inst}, {F.workers()} host processes", flush=True)
    return F.full_case(inst, N, L, LOG2_N1, LOG2_N2, KEY_FIRST, MSG_SEED, N_U, FLIP_SEED, K_FLIPS)


def first_mismatch(a, b):
    rows = np.nonzero((a != b).any(axis=1))[0]
    return int(rows[0]) if rows.size else None


@pytest.mark.parametrize("inst", [1, 0])
def test_full_aver_and_every_entry(P, gpu, inst):
    torch, ctx = gpu
    c = case_for(inst)
    assert c.aver_honest and not c.aver_corrupt
    params = P.make_params(inst, LOG2_N1, LOG2_N2)
    d = torch.from_numpy(c.msgs).cuda()
    print(f"inst {inst}: aver", flush=True)
    acc, e = P.poslo_aver(ctx, params, c.pk, P.make_msgs(d), c.ds, c.tag)
    assert acc is True and int.from_bytes(e, "little") == c.e
    eg, xg = P.poslo_ekeys(ctx, params, P.make_msgs(d), c.ds)
    eg, xg = eg.cpu().numpy(), xg.cpu().numpy()
    assert first_mismatch(xg, c.x_t) is None, first_mismatch(xg, c.x_t)
    assert first_mismatch(eg, c.e_t) is None, first_mismatch(eg, c.e_t)
    dc = torch.from_numpy(c.cmsgs).cuda()
    acc, e = P.poslo_aver(ctx, params, c.pk, P.make_msgs(dc), c.ds, c.tag)
    assert acc is False and int.from_bytes(e, "little") == c.e_corrupt


@pytest.mark.parametrize("inst", [1, 0])
def test_full_distill_and_sebver(P, gpu, inst):
    torch, ctx = gpu
    c = case_for(inst)
    assert c.invalid == sorted(e for e, _ in c.plan)
    params = P.make_params(inst, LOG2_N1, LOG2_N2)
    dm = torch.from_numpy(c.cmsgs).cuda()
    dsig = torch.from_numpy(np.ascontiguousarray(c.csigs).reshape(-1)).cuda()
    print(f"inst {inst}: distill", flush=True)
    ccd = P.poslo_distill(ctx, params, c.pk, P.make_msgs(dm), dsig, c.ds, N_U)
    assert ccd.invalid() == c.invalid
    assert ccd.valid_tag() == c.valid_tag
    umb, span = ccd.umbrellas()
    assert span == c.span and umb == c.umbrellas
    for k in (0, len(c.invalid) // 2, len(c.invalid) - 1):
        assert ccd.invalid_sig(k) == bytes(c.csigs[c.invalid[k]])
    m = P.make_msgs(dm)
    assert P.poslo_sebver(ctx, params, c.pk, m, ccd, "V") == [True]
    assert P.poslo_sebver(ctx, params, c.pk, m, ccd, "U") == [True] * N_U
    assert P.poslo_sebver(ctx, params, c.pk, m, ccd, "I") == [False] * len(c.invalid)


K_FLIP_EPOCHS = (N >> LOG2_N2) // 100


@pytest.mark.parametrize("inst", [1, 0])
def test_full_posloc(P, gpu, inst):
    import oracle_fullsize as F
    torch, ctx = gpu
    print(f"POSLO-C oracle over the full batch, inst {inst}", flush=True)
    c = F.full_case_c(inst, N, L, LOG2_N1, LOG2_N2, KEY_FIRST + 1, MSG_SEED, N_U, FLIP_SEED, K_FLIP_EPOCHS)
    assert c.aver_honest and not c.aver_corrupt
    assert c.invalid == sorted(i for i, _ in c.plan)
    params = P.make_params(inst, LOG2_N1, LOG2_N2)
    key = P.poslo_c_key_load(ctx, params, c.pk)
    d = torch.from_numpy(c.msgs).cuda()
    acc, e = P.poslo_c_aver(ctx, params, key, P.make_msgs(d), c.ds, c.s_total)
    assert acc is True and int.from_bytes(e, "little") == c.e
    dc = torch.from_numpy(c.cmsgs).cuda()
    k = N >> LOG2_N2
    cs = [c.cs_epochs[32 * i:32 * i + 32] for i in range(k)]
    from oracle import oracle as O
    acc, e = P.poslo_c_aver(ctx, params, key, P.make_msgs(dc), c.ds, O.posloc_agg_s(cs))
    assert acc is False and int.from_bytes(e, "little") == c.e_corrupt
    ccd = P.poslo_c_distill(ctx, params, key, P.make_msgs(dc), c.cs_epochs, c.ds, N_U)
    assert ccd.invalid() == c.invalid
    assert ccd.valid_tag() == c.valid_tag
    umb, span = ccd.umbrellas()
    assert span == c.span and umb == c.umbrellas
    m = P.make_msgs(dc)
    assert P.poslo_c_sebver(ctx, params, key, m, ccd, "V") == [True]
    assert P.poslo_c_sebver(ctx, params, key, m, ccd, "U") == [True] * N_U
    assert P.poslo_c_sebver(ctx, params, key, m, ccd, "I") == [False] * len(c.invalid)
