"""The gfx950 device code of every kernel keeps each store's data registers
untouched until the store has completed (see paper_1108_2473_amd/isa_check.py):
no vector write to a store's data registers before `s_waitcnt vmcnt(0)` or
the end of the kernel.  Compiles the sources to device assembly (CPU only)."""
import shutil

import pytest


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_no_store_data_overwrite():
    from paper_1108_2473_amd import isa_check
    findings = isa_check.check(jobs=5)
    assert findings == [], "\n".join(f"{f[0]} {f[1][:60]}: '{f[2]}' <- '{f[3]}'" for f in findings[:10])


def test_scanner_flags_the_pattern():
    """The scanner itself: an overwrite before the wait is flagged, one after it is not."""
    from paper_1108_2473_amd import isa_check
    bad = """_Zk: ; @_Zk
\tbuffer_store_dwordx4 v[0:3], v10, s[4:7], s18 offen
\tv_mul_f32_e32 v2, v49, v49
\ts_endpgm
"""
    good = """_Zk: ; @_Zk
\tbuffer_store_dwordx4 v[0:3], v10, s[4:7], s18 offen
\ts_waitcnt vmcnt(0)
\tv_mul_f32_e32 v2, v49, v49
\ts_endpgm
"""
    other = """_Zk: ; @_Zk
\tglobal_store_dwordx2 v[4:5], v[0:1], off
\tv_mad_i64_i32 v[0:1], s[6:7], s5, v6, v[48:49]
\ts_endpgm
"""
    assert len(isa_check.scan_asm(bad)) == 1
    assert isa_check.scan_asm(good) == []
    assert len(isa_check.scan_asm(other)) == 1
