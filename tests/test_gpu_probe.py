"""The measurement probes behind the bench line's ceilings (nbt_ig_probe_memory,
nbt_ig_probe_mfma): they read what they are said to read and count what they are said to do.

* stream: every 16-byte piece of the buffer, `count` passes; the xor of all sink words is the
  xor of the buffer's words for an odd pass count and zero for an even one;
* gather / quad gather: the positions follow the documented xorshift32 sequence (Marsaglia's
  13/17/5 shifts) per lane or per quad; the host replays it and the xors must agree;
* MFMA: deterministic sink, the stated FLOP count, argument checks.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_22588_amd as nbt
    ctx = nbt.Context(0)
    yield nbt, ctx
    ctx.close()


def _xor_all(a):
    return int(np.bitwise_xor.reduce(a.astype(np.uint32)))


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_stream_probe_reads_every_piece(env, passes):
    import torch
    nbt, ctx = env
    _note(f"stream probe, 64 KiB, {passes} passes")
    rng = np.random.default_rng(400 + passes)
    host = rng.integers(0, 2 ** 32, size=(1 << 14), dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(host.view(np.int32)).cuda()
    sink = nbt.binding.probe_memory(ctx, nbt.binding.PROBE_STREAM, buf, passes)
    got = _xor_all(sink.cpu().numpy().view(np.uint32))
    want = _xor_all(host) if passes % 2 else 0
    assert got == want


def _xorshift32(x):
    x = x ^ ((x << 13) & 0xFFFFFFFF)
    x = x ^ (x >> 17)
    x = x ^ ((x << 5) & 0xFFFFFFFF)
    return x


@pytest.mark.parametrize("group", [1, 4])
def test_gather_probes_follow_their_sequence(env, group):
    import torch
    nbt, ctx = env
    _note(f"gather probe, group {group}")
    words, loads = 1 << 12, 5
    rng = np.random.default_rng(410 + group)
    host = rng.integers(0, 2 ** 32, size=words, dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(host.view(np.int32)).cuda()
    kind = nbt.binding.PROBE_GATHER if group == 1 else nbt.binding.PROBE_QUAD_GATHER
    sink = nbt.binding.probe_memory(ctx, kind, buf, loads)
    lanes = 256 * nbt.binding._lib.nbt_ig_probe_sink_words(ctx.handle)
    gid = np.arange(lanes, dtype=np.uint64)
    h = ((gid // group) * np.uint64(2654435761) + np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF)
    h = np.where(h == 0, np.uint64(1), h)
    h = _xorshift32(h)
    mask = np.uint64(words - 1 if group == 1 else (words >> 2) - 1)
    sub = (gid % np.uint64(256)) & np.uint64(3)
    x = np.zeros(lanes, dtype=np.uint32)
    for _ in range(loads):
        h = _xorshift32(h)
        w = (h & mask) if group == 1 else (((h & mask) << np.uint64(2)) | sub)
        x ^= host[w.astype(np.int64)]
    assert _xor_all(sink.cpu().numpy().view(np.uint32)) == _xor_all(x)


@pytest.mark.parametrize("kind", [0, 1])
def test_mfma_probe(env, kind):
    import torch
    nbt, ctx = env
    _note(f"MFMA probe, kind {kind}")
    cu = ctx.info()["cu_count"]
    small = kind == nbt.binding.PROBE_MFMA_16X16X32_BF16
    chains, per = (16, 2 * 16 * 16 * 32) if small else (8, 2 * 32 * 32 * 16)
    for waves in (1, 2):
        s1, flops = nbt.binding.probe_mfma(ctx, kind, waves, 64)
        s2, _ = nbt.binding.probe_mfma(ctx, kind, waves, 64)
        torch.cuda.synchronize()
        assert torch.equal(s1[: cu * waves], s2[: cu * waves])
        assert flops == cu * waves * 4 * 64 * chains * per
    for bad in ((2, 1, 1), (kind, 0, 1), (kind, 9, 1), (kind, 1, 0)):
        with pytest.raises(nbt.NbtError) as e:
            nbt.binding.probe_mfma(ctx, *bad)
        assert e.value.status == nbt.binding.EINVAL
