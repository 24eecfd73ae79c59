"""The entry point that allocates nothing (gz_decompress_static), through the
C ABI on an MI355X: its output equals gz_decompress's (caller workspace) and
the source text, on two calls in a row on one GPU, the second with a smaller
input, and a plan whose workspace exceeds the static array is refused."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(b):
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda:0")


def test_static_workspace_matches_caller_workspace(orc):
    import paper_1905_07224_amd as gz

    L = gz.lib()
    inputs = [synth.fastq_like(4 << 20, 1), synth.word_stream(700 << 10, 2)]  # the second is smaller
    for k, raw in enumerate(inputs):
        comp = synth.gzip_member(raw, 6)
        _say("static workspace, call", k, len(raw), "bytes")
        d = _dev(comp)
        plan = gz.Plan(d, 0)
        assert plan.info.ws_bytes <= gz.GZ_SCRATCH_BYTES
        ref_out = torch.zeros(len(raw) + 64, dtype=torch.uint8, device="cuda:0")
        plan.launch(ref_out)
        r1 = plan.result()
        assert r1.status == 0
        want = ref_out[: r1.out_len].cpu().numpy().tobytes()
        tab1 = plan.chunk_table()
        out = torch.full((len(raw) + 64,), 0xAB, dtype=torch.uint8, device="cuda:0")
        st = torch.cuda.current_stream()
        rc = L.gz_decompress_static(plan._h, C.c_void_p(out.data_ptr()), out.numel(), C.c_void_p(st.cuda_stream))
        assert rc == 0, gz.lib().gz_strerror(rc)
        r2 = plan.result()
        assert r2.status == 0 and r2.out_len == r1.out_len == len(raw)
        got = out[: r2.out_len].cpu().numpy().tobytes()
        assert got == want == raw
        assert out[r2.out_len:].cpu().numpy().tolist() == [0xAB] * 64
        tab2 = plan.chunk_table()
        for key in ("start", "end", "len", "out_off"):
            assert np.array_equal(tab1[key], tab2[key]), key
        assert r2.crc32 == r1.crc32 == orc.crc32(raw)


def test_static_workspace_refuses_large_plans():
    import paper_1905_07224_amd as gz

    raw = synth.fastq_like(24 << 20, 3)
    comp = synth.gzip_member(raw, 6)
    plan = gz.Plan(_dev(comp), 0)
    assert plan.info.ws_bytes > gz.GZ_SCRATCH_BYTES
    out = torch.empty(len(raw), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(gz.GzError) as ei:
        plan.launch_static(out)
    assert ei.value.code == gz.GZ_E_CAPACITY
