"""The random-gather bandwidth probe reads what it states: lane s of quad q XORs the 16-byte
word s of every chunk its xorshift32 sequence draws.  The host replays the documented
sequence for every lane and compares the sinks exactly."""
import numpy as np
import pytest
import torch

from paper_2508_15522_amd import device as D, gridff as G
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def _expected(words, n_threads, iters, seed):
    """words: uint32 [n_chunks][16]; the XOR each lane accumulates."""
    n_chunks = words.shape[0]
    M = np.uint64(0xFFFFFFFF)
    q = np.arange(n_threads // 4, dtype=np.uint64)
    h = ((q * np.uint64(0x9E3779B9)) & M) ^ np.uint64(seed)
    h[h == 0] = np.uint64(0x6D2B79F5)
    acc = np.zeros((n_threads // 4, 4), np.uint32)
    lane_words = words.reshape(n_chunks, 4, 4)                      # [chunk][lane][word]
    for _ in range(iters):
        h ^= (h << np.uint64(13)) & M
        h ^= h >> np.uint64(17)
        h ^= (h << np.uint64(5)) & M
        c = ((h * np.uint64(n_chunks)) >> np.uint64(32)).astype(np.int64)
        sel = lane_words[c]                                         # [quad][lane][word]
        acc ^= sel[..., 0] ^ sel[..., 1] ^ sel[..., 2] ^ sel[..., 3]
    return acc.reshape(-1)


@pytest.mark.parametrize("n_chunks,iters", [(1000, 7), (4096, 8)])
def test_gather_probe_reads_the_documented_chunks(n_chunks, iters):
    D.require_gpu()
    announce(f"gather probe {n_chunks} chunks, {iters} gathers per lane")
    rng = np.random.default_rng(n_chunks)
    host = rng.integers(0, 2 ** 32, size=(n_chunks, 16), dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(host.view(np.int32).reshape(-1)).cuda()
    n_threads = 2048
    sink = torch.empty(n_threads, dtype=torch.int32, device="cuda")
    G.gather_probe(buf, n_threads, iters, 12345, sink)
    torch.cuda.synchronize()
    got = sink.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, _expected(host, n_threads, iters, 12345))


def test_gather_probe_rejects_invalid_arguments():
    D.require_gpu()
    buf = torch.zeros(64 * 16, dtype=torch.int32, device="cuda")
    sink = torch.empty(256, dtype=torch.int32, device="cuda")
    for n_threads, iters in ((100, 4), (256, 0)):
        with pytest.raises(G.GffError):
            G.gather_probe(buf, n_threads, iters, 1, sink)
    with pytest.raises(G.GffError):                                  # not 16-byte aligned
        G.gather_probe(buf[1:-3], 256, 4, 1, sink)
    with pytest.raises(G.GffError):                                  # not a multiple of 64 bytes
        G.gather_probe(buf[:-4], 256, 4, 1, sink)
