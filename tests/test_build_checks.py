"""Host-side checks the build applies to the compiled device code."""
import pytest

from paper_2512_15187_amd import build


def _asm(tmp_path, text):
    p = tmp_path / "k-hip-amdgcn-amd-amdhsa-gfx950.s"
    p.write_text(text)
    return str(p)


def test_m0_only_set_for_lds_loads(tmp_path):
    ok = ("\ts_mov_b32 m0, s16\n\tbuffer_load_dwordx4 v82, s[44:47], 0 offen lds\n\tv_add_u32 v1, v2, v3\n"
          "\ts_mov_b32 m0, vcc_lo\n\tbuffer_load_dword v3, s[8:11], 0 offen lds\n")
    build.check_m0(_asm(tmp_path, ok))


@pytest.mark.parametrize("text", [
    "\ts_mov_b32 m0, s16\n\tv_add_u32 v1, v2, v3\n",                 # M0 set, no load follows
    "\ts_add_i32 m0, s1, s2\n\tbuffer_load_dword v1, s[0:3], 0 offen lds\n",   # set by the compiler
    "\tv_movrels_b32 v1, v2\n\ts_mov_b32 m0, s3\n\tds_gws_init v0\n",   # another user of M0
])
def test_m0_other_uses_fail(tmp_path, text):
    with pytest.raises(RuntimeError):
        build.check_m0(_asm(tmp_path, text))
