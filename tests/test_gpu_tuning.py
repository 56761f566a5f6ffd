"""Launch-shape invariance: every blind-rotation workgroup shape and key-switch form gives the
same ciphertexts bit for bit (integer arithmetic), equal to the oracle's; the autotuner keeps
valid choices and round-trips them through its cache file."""
import json

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2010_09410_amd import VspError, client
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
SHAPES = [(4, 0), (4, 1), (4, 2), (8, 0), (8, 1), (8, 2), (3, 0), (3, 2), (32, 2), (32, 0), (8, 3), (32, 3),
          (33, 2), (33, 3), (33, 0)]


def batch(keys, B, seed):
    cfg = W.gate_batch(seed, B)
    g = W.rng(900 + seed)
    cfg["ops"] = g.integers(0, 9, B).astype(np.uint8)  # all nine opcodes, NOT included
    in0 = client.tlwe_encrypt_bits(keys["s0"], cfg["bits0"], *cfg["enc0"])
    in1 = client.tlwe_encrypt_bits(keys["s0"], cfg["bits1"], *cfg["enc1"])
    return cfg, in0, in1


@pytest.mark.parametrize("B,sample", [(37, None), (300, 12)])
def test_every_launch_shape_bit_identical(gpu, keys, B, sample):
    """B=37 and B=300 are ragged for 4- and 8-gate workgroups, 16-gate key-switch tiles and
    32-gate matrix-core tiles; shape 3 runs each gate on three waves, 32 on the matrix cores, 33
    on the matrix cores split by sub-product and row group."""
    _, saved_t = gpu.tuning(B)
    cfg, in0, in1 = batch(keys, B, 31 + B)
    d0, d1, dops = gpu.tensor(in0), gpu.tensor(in1), gpu.tensor(cfg["ops"])
    outs = []
    try:
        for w, t in SHAPES:
            gpu.set_tuning(B, w, t)
            assert gpu.tuning(B) == (w, t)
            outs.append(to_host(gpu.gates(dops, d0, d1)))
    finally:
        gpu.set_tuning(B, 0, saved_t)
    for o, shape in zip(outs[1:], SHAPES[1:]):
        np.testing.assert_array_equal(o, outs[0], err_msg=f"shape {shape}")
    idx = np.arange(B) if sample is None else np.unique(np.r_[0, B - 1, W.rng(7).choice(B, sample, replace=False)])
    ref = oracle.gates(keys["bk"], keys["ksk"], cfg["ops"][idx], in0[idx], in1[idx])
    np.testing.assert_array_equal(outs[0][idx], ref)


def test_tuning_set_rejects_unknown_shapes(gpu):
    with pytest.raises(VspError):
        gpu.set_tuning(64, 6, 0)
    with pytest.raises(VspError):
        gpu.set_tuning(64, 2, 0)
    with pytest.raises(VspError):
        gpu.set_tuning(64, 8, 4)
    # split-form workgroup counts: the valid ones round-trip, others are refused
    prev = gpu.set_split_groups(300, 2)
    try:
        for g in (1, 3, 6, 12, 24, -1, -2, -3, -6, -12, -24, 0):
            assert gpu.set_split_groups(300, g) in (1, 2, 3, 6, 12, 24, -1, -2, -3, -6, -12, -24, 0)
        assert gpu.set_split_groups(300, 2) == 0
        for bad in (4, 5, 7, -5, 48, -48, -4):
            with pytest.raises(VspError):
                gpu.set_split_groups(300, bad)
        assert gpu.set_split_groups(300, 2) == 2      # a refused value changes nothing
    finally:
        gpu.set_split_groups(300, prev)


BUCKETS = (1, 16, 64, 256, 1024, 2048, 4096)


def model_choice(entry, B):
    """The launch rule: fewest rounds x round time for the one-wave-per-gate forms and the
    matrix-core form, the interpolated per-bucket time for the split matrix-core form (ties:
    the 8-gate workgroup, then the order 4, 3, 32, 33)."""
    caps, ms, sms, at = entry["br_cap"], entry["br_round_ms"], entry["split_ms"], entry["split_at"]
    def split(B):
        b = next((i for i, k in enumerate(at) if B <= k), len(at) - 1)
        if B >= at[-1]:
            return sms[-1] * B / at[b]
        if b == 0:
            return sms[0]
        f = (B - at[b - 1]) / (at[b] - at[b - 1])
        return sms[b - 1] + f * (sms[b] - sms[b - 1])
    est = {s: -(-B // caps[s]) * ms[s] for s in range(4)}
    est[4] = split(B) * (1.03 if B > 1280 else 1.0)
    best = 1
    for s in (0, 2, 3, 4):
        if est[s] < est[best]:
            best = s
    return [4, 8, 3, 32, 33][best]


def test_autotune_model_and_cache_round_trip(gpu, tmp_path):
    saved = {b: gpu.tuning(b)[1] for b in BUCKETS}
    path = tmp_path / "tune.json"
    try:
        gpu.autotune(max_batch=64, cache_path=str(path))
        (key, entry), = json.loads(path.read_text()).items()
        assert key.startswith("gfx950")
        assert entry["br_waves"] == [4, 8, 3, 32, 33] and list(entry["buckets"]) == list(BUCKETS)
        cap4, cap8, capw, capm, caps = entry["br_cap"]
        assert 256 <= cap4 < cap8 and capw >= 256 and capm >= cap8 and caps == 32
        assert all(ms > 0 for ms in entry["br_round_ms"]) and all(ms > 0 for ms in entry["split_ms"])
        assert all(g in (1, 2, 3, 6, 12, 24, -1, -2, -3, -6, -12, -24) for g in entry["split_groups"])
        assert all(t in (0, 1, 2, 3) for t in entry["ks_form"])
        for b, t in zip(BUCKETS, entry["ks_form"]):
            assert gpu.tuning(b)[1] == t
        # the measured entry, read back from the file, picks what the rule says at every size
        gpu.autotune(max_batch=64, cache_path=str(path))
        for B in (1, 16, 40, 64, 200, 256, 700, 1024, 1200, 1500, 1900, 2048, 3000, 4096, 5000):
            assert gpu.tuning(B)[0] == model_choice(entry, B), B
        # edited entries for this GPU are read back and followed
        big = [100.0] * 13
        assert entry["split_at"] == [1, 16, 64, 256, 512, 768, 1024, 1280, 1536, 1792, 2048, 3072, 4096]
        for ms, sms, small, large in (([1.0, 100.0, 100.0, 100.0, 100.0], big, 4, 4),
                                      ([100.0, 1.0, 100.0, 100.0, 100.0], big, 8, 8),
                                      ([1.0, 1.5, 100.0, 100.0, 100.0], big, 4, 8),
                                      ([100.0, 100.0, 1.0, 100.0, 100.0], big, 3, 3),
                                      ([100.0, 100.0, 100.0, 1.0, 100.0], big, 32, 32),
                                      ([100.0, 100.0, 100.0, 100.0, 100.0], [0.001] * 13, 33, 33),
                                      ([100.0, 1.0, 100.0, 100.0, 100.0], [0.5] * 7 + [1000.0] * 6, None, None)):
            entry["br_round_ms"] = ms
            entry["split_ms"] = sms
            path.write_text(json.dumps({key: entry}))
            gpu.autotune(max_batch=64, cache_path=str(path))
            for B, want in ((cap4, small), (cap4 + 1, large)):
                assert gpu.tuning(B)[0] == (want if want is not None else model_choice(entry, B)), (ms, sms, B)
    finally:
        for b, t in saved.items():
            gpu.set_tuning(b, 0, t)


def test_autotune_cache_read_back_with_every_key_switch_form(gpu, tmp_path):
    """A cache entry naming every key-switch form (the matrix-core form 3 included) is read
    back as written, without measuring again (the file is left as it was); an entry written for
    another list of blind-rotation forms is ignored, measured again and rewritten."""
    saved = {b: gpu.tuning(b)[1] for b in BUCKETS}
    path = tmp_path / "tune.json"
    try:
        gpu.autotune(max_batch=64, cache_path=str(path))
        (key, entry), = json.loads(path.read_text()).items()
        entry["ks_form"] = [3, 2, 3, 1, 3, 0, 3]
        text = json.dumps({key: entry})
        path.write_text(text)
        gpu.autotune(max_batch=64, cache_path=str(path))
        assert path.read_text() == text
        for b, t in zip(BUCKETS, entry["ks_form"]):
            assert gpu.tuning(b)[1] == t
        shapes = list(entry["br_waves"])
        entry["br_waves"] = shapes[:-1] + [shapes[-1] + 1]
        path.write_text(json.dumps({key: entry}))
        gpu.autotune(max_batch=64, cache_path=str(path))
        assert json.loads(path.read_text())[key]["br_waves"] == shapes
    finally:
        for b, t in saved.items():
            gpu.set_tuning(b, 0, t)


def test_profile_sampling(gpu, keys):
    """Kernel-time instrumentation: every launch with on = 1, every k-th launch of each kind
    with on = k, none after disabling; a negative setting is an argument error."""
    from paper_2010_09410_amd import _native as nv
    cfg, in0, in1 = batch(keys, 8, 7)
    d0, d1, dops = gpu.tensor(in0), gpu.tensor(in1), gpu.tensor(cfg["ops"])
    out = gpu.gates(dops, d0, d1)
    try:
        for period, want in ((1, 8), (3, 3), (8, 1)):
            nv.vsp_profile_enable(gpu.handle, period)
            for _ in range(8):
                gpu.gates(dops, d0, d1, out=out)
            ms, n = nv.vsp_profile_read(gpu.handle, 0)
            assert n == want and ms > 0, (period, n, ms)
        nv.vsp_profile_enable(gpu.handle, 0)
        gpu.gates(dops, d0, d1, out=out)
        assert nv.vsp_profile_read(gpu.handle, 0)[1] == 0
        with pytest.raises(VspError):
            nv.vsp_profile_enable(gpu.handle, -1)
    finally:
        nv.vsp_profile_enable(gpu.handle, 0)


def test_profile_ignores_captured_and_server_launches(gpu, keys):
    """With profiling on, a circuit created (its levels captured into a graph) and run, and a
    server run on its worker thread, record no events: only eager calls on the caller's thread
    are instrumented; an eager gate call afterwards is."""
    from paper_2010_09410_amd import _native as nv
    c = W.small_circuit(seed=1300, levels=3, wmin=4, wmax=40, ninputs=16)
    x = client.tlwe_encrypt_bits(keys["s0"], c["bits"], *c["enc"])
    try:
        nv.vsp_profile_enable(gpu.handle, 1)
        circ = gpu.circuit(c["gates"], c["ninputs"])
        circ.run(gpu.tensor(x))
        gpu.sync()
        circ.close()
        srv = gpu.server(mem_budget_bytes=16 << 20, max_batch=64)
        t = srv.submit(c["gates"], c["ninputs"], x)
        import time
        t0 = time.time()
        while not srv.poll(t, c["ninputs"] + len(c["gates"]))[0]:
            assert time.time() - t0 < 120
            time.sleep(0.005)
        srv.close()
        for which in range(4):
            assert nv.vsp_profile_read(gpu.handle, which)[1] == 0, which
        cfg, in0, in1 = batch(keys, 8, 7)
        gpu.gates(gpu.tensor(cfg["ops"]), gpu.tensor(in0), gpu.tensor(in1))
        assert nv.vsp_profile_read(gpu.handle, 0)[1] == 1
    finally:
        nv.vsp_profile_enable(gpu.handle, 0)
