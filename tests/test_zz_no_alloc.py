"""The allocation-free entry point xs21_power_spectrum_static (static device
scratch) against the workspace entry point xs21_power_spectrum on the same
fields, through the C-ABI: two calls in a row, the second on a smaller box,
then a box too large for the static scratch (rejected with a clear error)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

AMP = synth.reference_amplitude()


def test_static_scratch_power_spectrum_matches_workspace_form():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1501_06576_amd as xs
    xs.library()
    ctx = xs.Context(0, phys=xs.physics(pk_amp=AMP))
    specs = [(128, 250.0, 9.0, 15, 2), (64, 128.0, 8.0, 12, 1), (256, 250.0, 9.0, 15, 3)]
    boxes, hs = [], []
    for n, box, z, nb, seed in specs:
        d = synth.make_box(n, box, z, seed=seed, amp=AMP, dtype=np.float32)
        boxes.append(d)
        hs.append(ctx.add_box(d, box, z, nb))
    ctx.prepare("f32", max_walkers=1, max_plain_radii=40)
    # fields: 27 (1 + delta) and a field with structure on every scale, each once
    for k in range(2):
        for (n, box, z, nb, _), h, d in zip(specs[:2], hs[:2], boxes[:2]):
            f = (27.0 * (1.0 + d)) if k == 0 else (d * d - 0.3 * d)
            ft = torch.from_numpy(np.ascontiguousarray(f.astype(np.float32))).cuda()
            ref = ctx.power_spectrum(h, ft)
            got = ctx.power_spectrum_static(h, ft).cpu().numpy()
            same = bool(np.array_equal(got, ref))
            rel = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))
            print(f"[static pk] n={n} field {k}: bitwise equal {same}, max rel diff {rel:.2e}", flush=True)
            assert rel <= 1e-12
    # 256^3 FP32 needs about 76 MB of scratch: rejected, the context stays usable
    ft = torch.from_numpy(boxes[2]).cuda()
    with pytest.raises(xs.Xs21Error, match="static scratch holds"):
        ctx.power_spectrum_static(hs[2], ft)
    ref = ctx.power_spectrum(hs[1], torch.from_numpy(boxes[1]).cuda())
    got = ctx.power_spectrum_static(hs[1], torch.from_numpy(boxes[1]).cuda()).cpu().numpy()
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-12
    ctx.close()
