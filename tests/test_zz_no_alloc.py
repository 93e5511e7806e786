"""The allocation-free loss/gradient entry point (mdnp_loss_grad_noalloc)
against the allocating one (mdnp_loss_grad), through the C ABI.

Both run the same kernels in the same order, so their outputs must agree bit
for bit; the allocating entry point is itself checked against the oracle's
Section 5.1 risk in the parity tests.  Two calls in a row share the fixed
workspace, the second with fewer slots (and the first call's contents still
in the workspace); a request beyond the workspace is refused.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

ARG = -1


def _P():
    import paper_2505_08491_amd as P
    return P


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def test_loss_grad_noalloc_matches_allocating_entry_point():
    P = _P()
    ctx = P.Context(0)
    insts = [synth.make_instance(900 + i, 16, n_segments=s, elems_per_segment=4, radius=0.008, beta=1.0)
             for i, s in enumerate((10, 5, 7))]
    S = P.System(ctx, insts, vec_dtype="f32")
    n3d = S.n3d
    rng = np.random.default_rng(17)
    for call, n_slots in enumerate((12, 5)):
        print(f"call {call}: {n_slots} slots of {n3d} unknowns", flush=True)
        slots = rng.integers(0, len(insts), n_slots).astype(np.int32)
        r = np.stack([synth.fast_normal(100 * call + k, n3d) for k in range(n_slots)])
        r /= np.linalg.norm(r, axis=1, keepdims=True)
        u = rng.normal(size=(n_slots, n3d)) * 1e-2
        inst_d, r_d, u_d = _dev(slots, torch.int32), _dev(r, torch.float32), _dev(u, torch.float32)
        loss_ref, du_ref = S.loss_grad(inst_d, r_d, u_d)
        du = torch.full_like(u_d, float("nan"))
        loss = torch.full((n_slots,), float("nan"), device="cuda", dtype=torch.float64)
        S.loss_grad_noalloc(inst_d, r_d, u_d, du, loss)
        torch.cuda.synchronize()
        assert torch.equal(loss, loss_ref), call
        assert torch.equal(du, du_ref), call
        assert bool(torch.isfinite(loss).all()) and float(loss.min()) > 0.0
    # a request beyond the fixed workspace (n_slots * (8 n3d + 512) > 32 MiB) is refused before any launch
    big = (32 << 20) // (8 * n3d + 512) + 1
    inst_d = torch.zeros(big, device="cuda", dtype=torch.int32)
    r_d = torch.zeros(big, n3d, device="cuda")
    du = torch.zeros_like(r_d)
    loss = torch.zeros(big, device="cuda", dtype=torch.float64)
    with pytest.raises(P.MdnpError) as e:
        S.loss_grad_noalloc(inst_d, r_d, r_d, du, loss)
    assert e.value.status == ARG
    assert "fixed workspace" in str(e.value)
    S.free()
    ctx.close()
