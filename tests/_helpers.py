"""Helpers shared by the GPU parity tests: read-back of the library's device buffers
and the comparison rules against the oracle."""
import numpy as np

IMG_TOL = 1e-4          # max-abs on pixels without a near-threshold evaluation
FLAGGED_TOL = 1e-2      # pixels the oracle flags (alpha near 1/255, T near 1e-4, power near 0)


def decode_record(st, n):
    """Splat record (n, 12) -> dict like the oracle's projection (valid where count > 0)."""
    rec = st.rec[: n * 12].view(n, 12).cpu().numpy()
    count = st.count[:n].cpu().numpy().view(np.uint32).astype(np.int64)
    r0 = rec[:, 10].view(np.uint32)
    r1 = rec[:, 11].view(np.uint32)
    rect = np.stack([r0 & 0xFFFF, r0 >> 16, r1 & 0xFFFF, r1 >> 16]).astype(np.int32)
    rect[:, count == 0] = 0
    return {"m": rec[:, 0:2].T.copy(), "conic": np.stack([rec[:, 2], rec[:, 3], rec[:, 4]]),
            "amax": rec[:, 5].copy(), "rgb": rec[:, 6:9].T.copy(), "depth": rec[:, 9].copy(),
            "rect": rect, "count": count.astype(np.int32), "n": n}


def read_bins(st):
    ni = int(st.num_inst.item())
    I = min(ni, st.capacity)
    keys = st.keys[:I].cpu().numpy().view(np.uint64)
    vals = st.values[:I].cpu().numpy().view(np.uint32)
    ranges = st.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    return {"keys": keys, "values": vals, "ranges": ranges, "I": ni}


def assert_projection_equal(gpu, orc, rgb_rtol=2e-6, amax_rtol=2e-6, near=None):
    """Integer decisions and FP-contract quantities bit-exact; continuous values close.
    near (optional): (scene, cam, t) of the frame; on a mismatch of a decision the message
    then gives the oracle's FP64 count of Gaussians within 1e-5 of a decision threshold
    (oracle.near_decisions) and whether the mismatching ones are among them."""
    def why(bad):
        if near is None:
            return bad[:10]
        import oracle

        n, idx = oracle.near_decisions(*near)
        return bad[:10], f"{n} Gaussians within 1e-5 of a decision; mismatches among them: " \
                         f"{np.isin(bad, idx).sum()} of {bad.size}"

    bad = np.nonzero(gpu["count"] != orc["count"])[0]
    assert bad.size == 0, why(bad)
    act = orc["count"] > 0
    bad = np.nonzero(np.any(gpu["rect"] != orc["rect"], axis=0) & act)[0]
    assert bad.size == 0, why(bad)
    assert np.array_equal(gpu["depth"][act].view(np.uint32), orc["depth"][act].view(np.uint32))
    assert np.array_equal(gpu["m"][:, act].view(np.uint32), orc["m"][:, act].view(np.uint32))
    assert np.array_equal(gpu["conic"][:, act].view(np.uint32), orc["conic"][:, act].view(np.uint32))
    np.testing.assert_allclose(gpu["amax"][act], orc["amax"][act], rtol=amax_rtol, atol=1e-12)
    np.testing.assert_allclose(gpu["rgb"][:, act], orc["rgb"][:, act], rtol=rgb_rtol, atol=2e-6)


def assert_bins_equal(gpu, orc):
    assert gpu["I"] == orc["I"]
    assert np.array_equal(gpu["keys"], orc["keys"])
    assert np.array_equal(gpu["values"], orc["values"])
    # a non-empty tile's [start, end) is unique; an empty tile only needs start == end
    g, o = gpu["ranges"].astype(np.int64), orc["ranges"].astype(np.int64)
    ne = o[:, 1] > o[:, 0]
    assert np.array_equal(g[ne], o[ne])
    assert np.all(g[~ne, 0] == g[~ne, 1])


def compare_images(img, final_T, n_contrib, res, tol=IMG_TOL):
    """img (3,H,W) float32 from the GPU vs the oracle blend result.  Returns stats."""
    flagged = (res["flags"] & 7) > 0  # bit 8 (alpha at the 0.99 clamp) only matters for gradients
    d = np.abs(img.astype(np.float64) - res["img"]).max(axis=0)
    ok = ~flagged
    stats = {"max_abs_unflagged": float(d[ok].max()) if ok.any() else 0.0,
             "max_abs_flagged": float(d[flagged].max()) if flagged.any() else 0.0,
             "n_flagged": int(flagged.sum()), "n_pixels": int(d.size)}
    assert stats["max_abs_unflagged"] <= tol, stats
    assert stats["max_abs_flagged"] <= FLAGGED_TOL, stats
    if n_contrib is not None:
        assert np.array_equal(n_contrib[ok], res["n_contrib"][ok]), stats
        np.testing.assert_allclose(final_T[ok], res["final_T"][ok], rtol=2e-4, atol=1e-7)
    return stats
