"""v-way stable partition (partition3 for v = 3) on the GPU, bit-exact
against the CPU oracle: keys, indices and class sizes."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


def run_both(x, v, kind, s=(0.0, 0.0, 0.0), cls=None, idx_dtype=torch.int64):
    print(f"[partv] n={len(x)} v={v} kind={kind} idx={idx_dtype}", flush=True)
    if kind == O.CLASS_MOD:
        c = P.Classes.mod(v)
    elif kind == O.CLASS_THRESH:
        c = P.Classes.thresholds(*s[: v - 1])
    else:
        c = P.Classes.from_bytes(torch.from_numpy(cls).to(DEV), v)
    ok, oi, cnt = P.partition_v(torch.from_numpy(x).to(DEV), c, idx_dtype=idx_dtype)
    ys, idx, counts = O.partition_v(x, v, kind, tuple(s), cls)
    assert np.array_equal(cnt.cpu().numpy(), counts)
    gi = oi.cpu().numpy().astype(np.int64)
    assert np.array_equal(gi, idx), f"first idx mismatch at {np.argmax(gi != idx)}"
    assert np.array_equal(ok.cpu().numpy().view(np.uint32), ys.view(np.uint32))


@pytest.mark.parametrize("v", [2, 3, 4])
@pytest.mark.parametrize("n", [0, 1, 3, 5, 1023, 4096, 4097, 12289, 100_003, (1 << 20) + 7])
def test_partition_v_sizes(n, v):
    g = np.random.default_rng(n + v)
    xi = (W.int_keys(n, 200 + n).astype(np.int64) - (1 << 30)).astype(np.int32)
    run_both(xi, v, O.CLASS_MOD)
    xf = g.random(n, dtype=np.float32)
    xf[::11] = np.nan
    s = tuple(np.sort(g.random(3)).astype(np.float32).tolist())
    run_both(xf, v, O.CLASS_THRESH, s, idx_dtype=torch.int32)
    cls = g.integers(0, 6, n).astype(np.uint8)
    run_both(xi, v, O.CLASS_BYTES, cls=cls)


def test_partition3_large_and_degenerate_classes():
    x = W.f32_uniform(1 << 24, 2)
    run_both(x, 3, O.CLASS_THRESH, (1 / 3, 2 / 3, 0.0), idx_dtype=torch.int32)
    run_both(x, 3, O.CLASS_THRESH, (-1.0, 2.0, 0.0))          # everything in class 1
    run_both(x, 3, O.CLASS_THRESH, (0.5, 0.5, 0.0))           # class 1 empty
    run_both(x, 4, O.CLASS_THRESH, (2.0, 3.0, 4.0))           # everything in class 0


def test_partition_v_rejects_bad_classes():
    x = torch.zeros(8, dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        P.partition_v(x, P.Classes.thresholds(0.5, 0.2))
    with pytest.raises(ValueError):
        P.partition_v(x, P.Classes(P.CLASS_MOD, 3))                 # modulus needs int32 keys
    with pytest.raises(ValueError):
        P.partition_v(x, P.Classes(P.CLASS_THRESH, 5, (0.1, 0.2, 0.3)))


def test_partition_v_multi_run_counting_ragged_tail():
    """n = 2^25 + 4097: 8194 tiles of 4096 elements, more than the 8192
    counting waves, so each counting wave owns two tiles and every tile's
    prefix is its offset inside the run plus the run's prefix; the last tile
    holds a single element."""
    n = (1 << 25) + 4097
    x = W.f32_uniform(n, 2)
    run_both(x, 3, O.CLASS_THRESH, (1 / 3, 2 / 3, 0.0), idx_dtype=torch.int32)
    xi = W.int_keys(n, 201)
    cls = np.random.default_rng(202).integers(0, 6, n).astype(np.uint8)
    run_both(xi, 4, O.CLASS_BYTES, cls=cls)
    n2 = (1 << 25) + 4099
    run_both(W.int_keys(n2, 203), 3, O.CLASS_MOD, idx_dtype=torch.int32)


def test_partition3_config_2e28():
    """partition3 of the 2^28 f32 uniform input (x < 1/3, x < 2/3, rest) with
    int32 indices, the launch the benchmark times: 65536 tiles, 8 per
    counting wave."""
    x = W.f32_uniform(W.FLAT_LARGE_N, W.FLAT_LARGE_SEED)
    run_both(x, 3, O.CLASS_THRESH, (1 / 3, 2 / 3, 0.0), idx_dtype=torch.int32)
