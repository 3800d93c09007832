"""Host logic of the batch streaming layout: a batch whose members'
distributions together exceed the in-place limit streams them between two
lattices; smaller batches leave each member's own choice."""
from paper_2308_05007_amd import autotune
from paper_2308_05007_amd import workloads as W


def _cfg(n, prec):
    return {"domain": {"n": (n, n, n), "precision": prec}, "walkers": {"n": 0}}


def test_the_sweep_streams_between_two_lattices():
    cfgs = [W.config_batch_member(i, steps=10) for i in range(64)]
    assert autotune.batch_streaming(cfgs) == 1


def test_small_batches_keep_each_members_layout():
    assert autotune.batch_streaming([_cfg(16, "fp64"), _cfg(32, "fp32")]) is None


def test_limit_counts_the_storage_bytes():
    # 19 distributions of 2^22 nodes: 304 MiB in FP32 (below 384 MiB), 608 MiB in FP64
    n = 1 << 22
    cfg = lambda prec: {"domain": {"n": (n, 1, 1), "precision": prec}, "walkers": {"n": 0}}
    assert autotune.batch_streaming([cfg("fp32")]) is None
    assert autotune.batch_streaming([cfg("fp64")]) == 1
    assert autotune.batch_streaming([cfg("fp16"), cfg("bf16")]) is None  # 304 MiB
    assert autotune.batch_streaming([cfg("fp16"), cfg("bf16"), cfg("fp16")]) == 1  # 456 MiB
    assert autotune.batch_streaming([cfg("fp32"), cfg("fp16")]) == 1


def test_signature_names_the_layout():
    big = [W.config_batch_member(i, steps=10) for i in range(64)]
    assert "|two|" in autotune.signature("batch", big)
    assert "|own|" in autotune.signature("batch", [_cfg(16, "fp32")])
