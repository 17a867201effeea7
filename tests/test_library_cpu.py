"""CPU-side checks of the HIP library: it loads without a GPU, exports every
symbol include/coralai.h declares, and its host-only entry points (sizes,
argument validation) behave as documented.  No compute call is made."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "coralai.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(coralai_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_2406_09654_amd import binding
    binding.lib()
    return binding


def test_library_exports_every_declared_symbol(B):
    syms = declared_symbols()
    assert len(syms) >= 20
    L = B.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(B.EXPORTED) == syms


def test_world_bytes_and_validation(B):
    from paper_2406_09654_amd.world import make_desc
    d = make_desc(64, 64)
    n = B.coralai_world_bytes(d)
    N = 64 * 64
    assert n > 2 * 37 * N + 41 * N          # two state buffers + the boundary record
    d3 = make_desc(4096, 4096, 3, 64, 1 << 17, 1)
    big = B.coralai_world_bytes(d3)
    assert big > (1 << 17) * 18 * 1024       # bf16 fragment tables
    for bad in [make_desc(0, 4), make_desc(4, 4, 4), make_desc(4, 4, 2, 48),
                make_desc(4, 4, 2, 32, 0), make_desc(4, 4, 2, 32, 4, 2),
                make_desc(4, 4, rho_invest=1.5), make_desc(4, 4, kappa_flow=float("nan"))]:
        assert B.coralai_world_bytes(bad) == 0


def test_create_rejects_small_arena_without_touching_gpu(B):
    from paper_2406_09654_amd.world import make_desc
    d = make_desc(16, 16)
    need = B.coralai_world_bytes(d)
    with pytest.raises(B.CoralaiError) as e:
        B.coralai_world_create(d, 0x1000, need - 1, 0)
    assert e.value.code == B.CORALAI_E_NOMEM
    with pytest.raises(B.CoralaiError) as e:
        B.coralai_world_create(make_desc(0, 16), 0x1000, need, 0)
    assert e.value.code == B.CORALAI_E_INVALID
    assert "width" in B.coralai_last_error()


def test_batch_bytes(B):
    assert B.coralai_batch_bytes(0) == 0
    assert B.coralai_batch_bytes(512) > 512 * 300


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_2406_09654_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "coralai_oracle" not in txt, f
