"""Code-generation guards on the lookup kernels (compiled here for gfx950,
no device needed): the lookups read LDS and global memory through their own
address spaces (no generic flat loads, which are slower and which the
compiler falls back to when a load's address may point to either), and no
kernel spills to scratch."""
import concurrent.futures
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2402_09222_amd"))
import build as B  # noqa: E402

SOURCES = ["xs_lookup_nuclide.hip", "xs_lookup_hash.hip", "xs_lookup_union.hip"]


def _asm(src, tmp):
    out = os.path.join(tmp, src + ".s")
    cmd = [B.HIPCC, *B.CXXFLAGS, "--cuda-device-only", "-S",
           os.path.join(B.CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    tmp = str(tmp_path_factory.mktemp("asm"))
    with concurrent.futures.ThreadPoolExecutor(3) as ex:
        texts = list(ex.map(lambda s: _asm(s, tmp), SOURCES))
    return dict(zip(SOURCES, texts))


def _kernels(text):
    """(name, body) of every kernel in an assembly listing."""
    out = []
    for m in re.finditer(r"^(_Z\S*k_lookup\S*):", text, re.M):
        end = text.find("s_endpgm", m.end())
        out.append((m.group(1), text[m.end():end]))
    return out


def test_lookup_kernels_use_no_flat_loads(asm):
    bad = [name for text in asm.values() for name, body in _kernels(text)
           if "flat_load" in body]
    assert not bad, bad


def test_lookup_kernels_do_not_spill(asm):
    for text in asm.values():
        for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", text):
            assert int(m.group(1)) == 0
