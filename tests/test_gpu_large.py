"""The largest configurations through the C ABI (needs an MI355X).

4 GiB of FASTQ-like text (read lengths 100 and 150) compressed at levels 1
and 9 from the same seed, and 2 GiB of the Zipf word stream at level 6, each
decoded in the launch configuration the benchmark times (library defaults).
The whole output must equal the generated text byte for byte (the text is
the ground truth of the encoder round trip that the oracle tests pin), and
the device's CRC-32 must equal the trailer's.  A full sequential gunzip of
these members would take minutes on the host, so the block chain is pinned
by sampling: the encoder records where each of its 64 MiB compression
segments begins (a block boundary whose output offset it knows), and for a
seeded sample of chunks the oracle decodes from the segment's first block to
the chunk's start.  It must stop exactly at that start, a block boundary,
with the device's output offset.  From there the oracle's pass 1 must give
the device's end bit and 16-bit symbols (decompress(C_i, w_hat_i) of
Section VI-C), and the chunk's resolved window must be the 32 KiB of text
before it.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NAMES = ["fastq_4GiB_L1", "fastq_4GiB_L9", "words_2GiB_L6"]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("name", NAMES)
def test_large_against_source_and_oracle(orc, name):
    import paper_1905_07224_amd as gz

    _say("generating", name)
    raw, comp, seg_bits = synth.workload(name, index=True)
    _say(name, len(raw), "bytes,", len(comp), "compressed,", len(seg_bits), "encoder segments")
    dev = torch.device("cuda:0")
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to(dev)
    plan = gz.Plan(d_comp, 0)
    out = torch.empty(len(raw), dtype=torch.uint8, device=dev)
    plan.launch(out)
    r = plan.result()
    _say(name, "status", r.status, "chunks", plan.n_chunks, "repairs", r.n_repairs, "retries", r.n_retries)
    assert r.status == 0 and r.out_len == len(raw)
    d_raw = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    assert torch.equal(out, d_raw)
    del d_raw
    trailer_crc = int.from_bytes(comp[-8:-4], "little")
    assert r.crc32 == trailer_crc
    tab = plan.chunk_table()
    start = tab["start"].astype(np.uint64)
    ne = np.nonzero(start != np.uint64(gz.NONE))[0]
    assert ne[0] == 0 and int(start[0]) == 8 * plan.info.payload_start
    ends = tab["end"][ne].astype(np.int64)
    assert np.array_equal(ends[:-1], start[ne][1:].astype(np.int64))
    assert (ends[-1] + 7) // 8 + 8 == len(comp)
    offs = tab["out_off"][ne].astype(np.int64)
    lens = tab["len"][ne].astype(np.int64)
    assert np.array_equal(offs[1:], np.cumsum(lens)[:-1]) and int(lens.sum()) == len(raw)
    rng = np.random.default_rng(11)
    sample = sorted(set([int(ne[1]), int(ne[-1])] + [int(x) for x in rng.choice(ne[1:], 4, replace=False)]))
    segs = np.asarray(seg_bits, dtype=np.int64)
    for j in sample:
        k = int(np.nonzero(ne == j)[0][0])
        s, e, off = int(start[j]), int(ends[k]), int(offs[k])
        q = int(np.searchsorted(segs, s, side="right")) - 1
        _say(name, "chunk", j, "bits", s, e, "from encoder segment", q)
        # from the encoder's block boundary the oracle reaches the chunk start
        pre = orc.symbolic(comp, int(segs[q]), s, first=(q == 0))
        assert pre.status == orc.OK and pre.end_bit == s, f"chunk {j}: start off the block chain"
        assert q * synth.SEGMENT_BYTES + pre.sym.size == off
        del pre
        sr = orc.symbolic(comp, s, e, first=False)
        assert sr.status == orc.OK and sr.end_bit == e
        L = int(lens[k])
        assert sr.sym.size == L
        dsym = plan.symbols(j, L).cpu().numpy().view(np.uint16)
        assert np.array_equal(dsym, sr.sym), f"symbols of chunk {j}"
        w = plan.window(j).cpu().numpy()
        v = min(off, 32768)
        assert w[32768 - v:].tobytes() == raw[off - v:off], f"window of chunk {j}"
