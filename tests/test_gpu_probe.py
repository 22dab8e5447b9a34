"""The streaming-read probe reads every word of the stored matrix exactly
once, in both modes and at every segment length (rows of 2000 bytes end
inside a segment; 4109 rows end inside a tile), and rejects bad arguments."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def P():
    import paper_2109_03709_amd as mod
    return mod


@pytest.fixture(scope="module")
def data():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P().lib()
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    x = torch.randn((4109, 1000), generator=g, device="cuda").to(torch.bfloat16)
    words = x.contiguous().view(torch.int16).cpu().numpy().view(np.uint32)
    return P().Data(x, P().BF16), int(np.bitwise_xor.reduce(words, axis=None))


@pytest.mark.parametrize("mode,seg", [(0, 128), (1, 128), (1, 256), (1, 512)])
def test_probe_reads_every_word_once(data, mode, seg):
    X, ref = data
    print(f"read probe: mode {mode} seg {seg}", flush=True)
    sink = P().read_probe(X, mode, seg)
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    assert int(got) == ref


def test_probe_rejects_bad_arguments(data):
    X, _ = data
    with pytest.raises(P().PPCAError) as e:
        P().read_probe(X, 2)
    assert e.value.code == -1
    with pytest.raises(P().PPCAError) as e:
        P().read_probe(X, 1, 64)
    assert e.value.code == -1
    with pytest.raises(P().PPCAError) as e:
        P().read_probe(X, 0, 128, torch.zeros(8, dtype=torch.int32, device="cuda"))
    assert e.value.code == -1
