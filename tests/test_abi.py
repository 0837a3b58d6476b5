"""CPU checks of the C ABI: the library loads and exports every function that
include/ftv.h declares; the ctypes structures match the C layout; host-side
argument validation runs without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftv.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ftv_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1405_2912_amd as ftv
    return ftv.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    import paper_1405_2912_amd.ftv as b
    assert sorted(b.EXPORTS) == names


def test_no_unexpected_exports():
    so = os.path.join(ROOT, "paper_1405_2912_amd", "libftv.so")
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T ftv_" in ln})
    assert exported == _declared()
    # nothing but the C ABI is visible: internal C++ symbols are local
    others = sorted({ln.split()[-1] for ln in out.splitlines()
                     if ln.split() and not ln.split()[-1].startswith("ftv_")})
    assert others == [], others[:10]


def _c_sizes():
    """sizeof/offsetof of the ABI structures, from the C compiler."""
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "ftv.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(ftv_tol), sizeof(ftv_stats),
         sizeof(ftv_vote_desc), sizeof(ftv_batch_cfg), sizeof(ftv_block_stats),
         sizeof(ftv_server_cfg), sizeof(ftv_request), sizeof(ftv_result), sizeof(ftv_server_stats),
         sizeof(ftv_sibling_info), sizeof(ftv_mm_check_result), sizeof(ftv_impl),
         sizeof(ftv_redundancy_cfg), sizeof(ftv_redundancy_report));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", offsetof(ftv_stats, verdict), offsetof(ftv_vote_desc, tol),
         offsetof(ftv_vote_desc, stats), offsetof(ftv_request, t_arrival_ns), offsetof(ftv_request, ready),
         offsetof(ftv_sibling_info, readers), offsetof(ftv_mm_check_result, blocks),
         offsetof(ftv_redundancy_cfg, tol), offsetof(ftv_redundancy_report, seconds));
  return 0;
}
'''
    import tempfile
    d = tempfile.mkdtemp()
    c = os.path.join(d, "s.c")
    open(c, "w").write(src)
    exe = os.path.join(d, "s")
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
    lines = subprocess.check_output([exe], text=True).split("\n")
    return [int(x) for x in lines[0].split()], [int(x) for x in lines[1].split()]


def test_ctypes_layout_matches_c():
    import paper_1405_2912_amd.ftv as b
    sizes, offs = _c_sizes()
    mine = [ctypes.sizeof(t) for t in (b.Tol, b.Stats, b.VoteDesc, b.BatchCfg, b.BlockStats,
                                       b.ServerCfg, b.Request, b.Result, b.ServerStats,
                                       b.SiblingInfo, b.MMCheckResult, b.Impl, b.RedundancyCfg,
                                       b.RedundancyReport)]
    assert mine == sizes
    assert [b.Stats.verdict.offset, b.VoteDesc.tol.offset, b.VoteDesc.stats.offset,
            b.Request.t_arrival_ns.offset, b.Request.ready.offset, b.SiblingInfo.readers.offset,
            b.MMCheckResult.blocks.offset, b.RedundancyCfg.tol.offset,
            b.RedundancyReport.seconds.offset] == offs


def test_host_validation_without_gpu(lib):
    """Calls that fail validation return before touching the device."""
    import paper_1405_2912_amd.ftv as b
    assert lib.ftv_vote(None, None, None) == b.E_INVALID
    assert lib.ftv_vote_batch(None, None, 0, None) == b.E_INVALID
    assert b"context" in lib.ftv_last_error()
    cfg = b.ServerCfg(0, 0, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.ftv_server_create(ctypes.byref(cfg), ctypes.byref(h)) == b.E_INVALID
    assert lib.ftv_now_ns() > 0
    assert lib.ftv_version().startswith(b"ftv")


def test_product_path_does_not_use_the_oracle():
    """Neither the binding nor the library references the oracle."""
    for path in ("paper_1405_2912_amd/ftv.py", "paper_1405_2912_amd/__init__.py"):
        assert "oracle" not in open(os.path.join(ROOT, path)).read().replace("oracle is never", "")
    so = open(os.path.join(ROOT, "paper_1405_2912_amd", "libftv.so"), "rb").read()
    assert b"fto_" not in so and b"ftv_oracle" not in so
