"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function that include/ymine.h declares, and fails cleanly without a
device."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ymine.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ym_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1509_08639_amd import ymine
    if not os.path.exists(ymine.LIB_PATH):
        from paper_1509_08639_amd import build
        build.build()
    return ymine


def test_exports_every_declared_symbol(lib):
    L = lib.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lib.EXPORTS) == names


def test_version_and_error_string(lib):
    L = lib.lib()
    assert L.ym_version().startswith(b"ymine")
    assert L.ym_last_error() is not None


def test_no_device_is_a_clean_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(lib.YmError) as e:
        lib.Context(0)
    assert e.value.code == lib.YM_EDEVICE


def test_no_oracle_in_product():
    """The product (package + C sources) never references the oracle."""
    pkg = os.path.join(ROOT, "paper_1509_08639_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                t = open(os.path.join(dp, f)).read()
                assert "oracle" not in t.lower(), f


def test_pair_size_limits_on_the_host(lib):
    """Pairs whose score block would need 32-bit offsets of 2^31 or more (the
    similarity kernels' addressing) or documents of more than 2^22 sentences
    are rejected before any device work; the check needs no device."""
    lib.check_pair(0, 0)
    lib.check_pair(40000, 40000)  # about 1.6e9 score slots
    lib.check_pair(1 << 22, 100)
    for n, m in [(50000, 50000), (46341, 46341), ((1 << 22) + 1, 1), (1, (1 << 22) + 1), (-1, 5)]:
        with pytest.raises(lib.YmError) as e:
            lib.check_pair(n, m)
        assert e.value.code == lib.YM_EINVAL, (n, m)
