"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/gosh.h declares, and its host-only functions behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gosh.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:gosh_status|const char\*)\s+(gosh_\w+)\s*\(", txt, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("gosh_coarsen", "gosh_train", "gosh_prolong", "gosh_ctx_create", "gosh_update_batch",
                 "gosh_draw_samples", "gosh_epoch_schedule", "gosh_validate_csr"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2110_10049_amd import gosh as G
    L = C.CDLL(G.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(G.EXPORTS) == _declared()


def test_schedule_matches_oracle(orc):
    from paper_2110_10049_amd import gosh as G
    for e in (0, 1, 7, 200, 600, 1000):
        for p in (0.0, 0.1, 0.3, 0.5, 1.0):
            for D in (1, 2, 3, 6, 7, 11):
                assert G.gosh_epoch_schedule(e, p, D) == list(orc.epoch_schedule(e, p, D))


def test_schedule_rejects_bad_args():
    from paper_2110_10049_amd import gosh as G
    for args in ((10, -0.1, 3), (10, 1.1, 3), (-1, 0.3, 3)):
        with pytest.raises(G.GoshError) as ei:
            G.gosh_epoch_schedule(*args)
        assert ei.value.status == "E_INVALID_ARG"


def test_null_context_is_rejected():
    from paper_2110_10049_amd import gosh as G
    L = G.lib()
    assert L.gosh_sync(None) == 1
    assert L.gosh_train(None, None, 0, None, 0, 128, 1, 0.1, 3, 0, None) == 1
    assert L.gosh_last_error(None) == b"null context"
    assert L.gosh_ctx_destroy(None) == 0


def test_mlp_entry_points_reject_null():
    from paper_2110_10049_amd import gosh as G
    L = G.lib()
    n = C.c_int64()
    assert L.gosh_mlp_num_params(None, C.byref(n)) == 1
    assert L.gosh_mlp_destroy(None) == 0
    assert L.gosh_mlp_create(None, 128, 256, C.byref(C.c_void_p())) == 1
    assert L.gosh_mlp_train(None, None, 0, None, 0, 1, 32, 0.1, 0, None) == 1
    assert L.gosh_prolong(None, None, 0, None, None, 0, 128, None) == 1
