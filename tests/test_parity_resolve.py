"""CPU check of the parity tests' decision resolution (tests/parity_resolve.py):
given outputs computed with some of the oracle's flagged decisions taken the
other way (and float32-sized noise), it finds those decisions, and the
oracle rendered with them matches the outputs everywhere."""
import numpy as np
import torch

import oracle as O
from paper_2410_11419_amd import synth
from parity_resolve import resolve, describe


def _outputs(ref, W, H):
    f = lambda t: t.detach().numpy()  # noqa: E731
    return f(ref["T"]), {"final": f(ref["final"]), "S": f(ref["S"]), "Sh": f(ref["Sh"]), "R": f(ref["R"]),
                         "T_final": f(ref["T_final"])}


def test_resolution_recovers_flipped_decisions():
    sc, cam, light = synth.scene_small()
    k = O.Consts()
    ref0 = O.render(sc, cam, light, k)
    lk = torch.unique(ref0["amb_light_keys"]).tolist()
    ck = torch.unique(ref0["amb_cam_keys"]).tolist()
    sk = torch.unique(ref0["amb_stop_keys"]).tolist()
    assert lk and ck
    # the "GPU" takes every flagged light and camera decision the other way
    alt = O.render(sc, cam, light, k, light_flips=lk, cam_flips=ck, cam_stop_flips=sk)
    T_alt, px_alt = _outputs(alt, cam.width, cam.height)
    rng = np.random.default_rng(0)
    T_alt = T_alt + rng.normal(0, 1e-7, T_alt.shape)
    ref, info = resolve(sc, cam, light, k, None, None, T_alt, px_alt)
    print(describe(info))
    assert not info["unresolved_T"].any() and not info["unresolved_px"].any()
    assert np.abs(ref["T"].detach().numpy() - T_alt).max() < 1e-6
    for key in ("final", "S", "Sh", "R", "T_final"):
        assert np.abs(ref[key].detach().numpy() - px_alt[key]).max() < 1e-12, key
    # against the unflipped oracle the same outputs differ beyond the tolerance
    assert np.abs(ref0["T"].detach().numpy() - T_alt).max() > 1e-4
    # and outputs that follow the oracle's own decisions resolve to no flips
    T0, px0 = _outputs(ref0, cam.width, cam.height)
    _, info0 = resolve(sc, cam, light, k, None, None, T0, px0)
    assert info0["light_flipped"] == 0 and info0["cam_flipped"] == 0 and info0["stop_flipped"] == 0
