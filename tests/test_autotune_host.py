"""Host logic of the launch autotuner (no GPU): the stage plans tried per transform length, the
candidate lists and the cache key."""
import json
from types import SimpleNamespace

from paper_2004_13904_amd import autotune as T


def test_fft_plans_are_the_distinct_stage_sequences():
    # plan 0: radix-8 stages then the radix-4/2 stage; plan 1: that stage first; plan 2: radix-4
    # stages.  For a power of 8 plans 0 and 1 are the same sequence and only 0 is tried.
    for n in (8, 64, 512):
        assert T.fft_plans(n) == [0, 2]
    for n in (16, 32, 128, 256, 1024, 2048):
        assert T.fft_plans(n) == [0, 1, 2]


def _op(nfft, nz, batch_max):
    return SimpleNamespace(nfft=nfft, nz=nz, batch_max=batch_max, dtype="torch.float32")


def test_candidates_cover_every_tuning_key():
    op = _op((512, 256), 20, 48)
    c = T.candidates(op, batched=False)
    assert c["fft_plan_x"] == [0, 2] and c["fft_plan_y"] == [0, 1, 2]
    assert c["lg_G"] == c["lg_GT"] == [1, 2, 3, 4, 5, 8, 10, 20]
    assert c["row_tile"] == [0, 1, 2, 3, 4]
    assert "batch" not in c and "col_batched" not in c
    cb = T.candidates(op, batched=True)
    assert cb["batch"] == [4, 8, 16, 32, 48]
    assert cb["col_batched"] == [2, 1, 0]
    # layer groups never exceed the layers
    assert T.candidates(_op((64, 64), 3, 16), batched=False)["lg_G"] == [1, 2, 3]


def test_cache_key_is_embedding_layers_width_and_dtype(tmp_path):
    op = _op((256, 128), 10, 64)
    assert T._key(op, 1) == "NX256:NY128:nz10:k1:torch.float32"
    assert T._key(op, 16) == "NX256:NY128:nz10:k16:torch.float32"
    # a cached choice is applied without timing anything
    cache = tmp_path / "tune.json"
    choice = {"lg_G": 2, "lg_GT": 4, "row_tile": 3, "fft_plan_x": 2, "fft_plan_y": 0}
    cache.write_text(json.dumps({T._key(op, 1): choice}))
    applied = {}

    class Op(SimpleNamespace):
        def set_tuning(self, **kw):
            applied.update(kw)

        @property
        def tuning(self):
            return dict(applied)

    x = SimpleNamespace(dim=lambda: 1)
    got = T.autotune(Op(nfft=(256, 128), nz=10, batch_max=64, dtype="torch.float32"), x, None, cache=str(cache))
    assert got == choice
