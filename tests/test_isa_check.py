"""The build's check for barriers inside loops with divergent exits.

Two hand-written assembly fragments in the form hipcc emits: a work loop whose
barrier sits in a loop that thread 0 leaves on its own (the shape that makes a
workgroup spin), and the same work loop with only a uniform exit.
"""

import sys
from pathlib import Path

sys.path.insert(0, str(Path(__file__).resolve().parents[1] / "paper_1704_02278_amd"))
import isa_check  # noqa: E402

BAD = """\
kern:                                   ; @kern
	s_load_dwordx2 s[0:1], s[4:5], 0x0
	s_branch .LBB0_2
.LBB0_1:                                ;   in Loop: Header=BB0_2 Depth=1
	s_or_b64 exec, exec, s[4:5]
	s_andn2_b64 exec, exec, s[50:51]
	s_cbranch_execz .LBB0_9
.LBB0_2:                                ; =>This Loop Header: Depth=1
                                        ;     Child Loop BB0_4 Depth 2
	s_and_saveexec_b64 s[4:5], s[48:49]
	global_atomic_add_x2 v[2:3], v37, v[2:3], s[20:21] offset:16 sc0
.LBB0_4:                                ;   Parent Loop BB0_2 Depth=1
                                        ; =>  This Loop Header: Depth=2
	ds_write_b32 v65, v37
	s_waitcnt lgkmcnt(0)
	s_barrier
	ds_read_b64 v[4:5], v37 offset:128
	s_cbranch_vccnz .LBB0_5
; %bb.3:                                ;   in Loop: Header=BB0_4 Depth=2
	s_mov_b64 s[4:5], s[48:49]
.LBB0_5:                                ;   in Loop: Header=BB0_4 Depth=2
	s_and_b64 s[4:5], exec, s[4:5]
	s_or_b64 s[60:61], s[4:5], s[60:61]
	s_andn2_b64 exec, exec, s[60:61]
	s_cbranch_execnz .LBB0_4
; %bb.6:                                ;   in Loop: Header=BB0_2 Depth=1
	s_branch .LBB0_1
.LBB0_9:
	s_endpgm
.Lfunc_end0:
"""

GOOD = """\
kern:                                   ; @kern
	s_load_dwordx2 s[0:1], s[4:5], 0x0
.LBB0_1:                                ; =>This Loop Header: Depth=1
                                        ;     Child Loop BB0_3 Depth 2
	s_waitcnt lgkmcnt(0)
	s_barrier
	ds_read_b64 v[4:5], v37 offset:128
	s_cbranch_vccnz .LBB0_9
.LBB0_3:                                ;   Parent Loop BB0_1 Depth=1
                                        ; =>  This Inner Loop Header: Depth=2
	global_load_dword v2, v[0:1], off
	s_or_b64 s[6:7], vcc, s[6:7]
	s_andn2_b64 exec, exec, s[6:7]
	s_cbranch_execnz .LBB0_3
; %bb.4:                                ;   in Loop: Header=BB0_1 Depth=1
	s_or_b64 exec, exec, s[6:7]
	s_and_saveexec_b64 s[4:5], s[48:49]
	global_atomic_add_x2 v[2:3], v37, v[2:3], s[20:21] offset:16 sc0
	s_or_b64 exec, exec, s[4:5]
	s_branch .LBB0_1
.LBB0_9:
	s_endpgm
.Lfunc_end0:
"""


def _check(text, tmp_path):
    f = tmp_path / "k.s"
    f.write_text(text)
    return isa_check.check_file(f)


def test_flags_barrier_loop_with_divergent_exit(tmp_path):
    got = _check(BAD, tmp_path)
    assert set(got) == {"kern"}
    assert got["kern"] == ["loop BB0_2 holds s_barrier and has a divergent exit",
                           "loop BB0_4 holds s_barrier and has a divergent exit"]


def test_accepts_uniform_exit_with_divergent_inner_loop(tmp_path):
    assert _check(GOOD, tmp_path) == {}


def test_divergent_loop_without_barrier_is_fine(tmp_path):
    assert _check(GOOD.replace("\ts_barrier\n", ""), tmp_path) == {}


def _descriptor(name, scratch, group=160):
    return f"""\
	.amdhsa_kernel {name}
		.amdhsa_group_segment_fixed_size {group}
		.amdhsa_private_segment_fixed_size {scratch}
		.amdhsa_kernarg_size 304
	.end_amdhsa_kernel
"""


def test_flags_a_kernel_that_spills_to_scratch(tmp_path):
    got = _check(GOOD + _descriptor("kern", 0) + _descriptor("spilly", 64), tmp_path)
    assert got == {"spilly": ["uses 64 bytes of scratch per lane (register spill)"]}


def test_scratch_sizes_read_from_every_descriptor(tmp_path):
    f = tmp_path / "k.s"
    f.write_text(_descriptor("a", 0) + _descriptor("b", 8) + _descriptor("c", 0))
    assert isa_check.scratch_sizes(f.read_text().splitlines()) == {"a": 0, "b": 8, "c": 0}


def test_scan_kernels_must_have_no_static_lds(tmp_path):
    scan = "_ZN4glop6detail16glop_scan_kernelILi1ELb1ELi4ELb1ELi8ELb0EEEvNS0_10ScanParamsE"
    emit = "_ZN4glop6detail16glop_emit_kernelILi1ELb1ELi4ELb1ELi8ELb0EEEvNS0_10ScanParamsENS0_10EmitParamsE"
    ok = _check(_descriptor(scan, 0, group=0) + _descriptor(emit, 0, group=37000), tmp_path)
    assert ok == {}
    bad = _check(_descriptor(scan, 0, group=16), tmp_path)
    assert bad == {scan: ["has 16 bytes of static LDS (its tables must start at address 0)"]}


# A walk loop whose last LDS operation is an atomic add, exiting straight into
# the barrier after which another wave reads the sum (the shape in which the
# compiler left out the wait): the barrier must be preceded by lgkmcnt(0).
UNWAITED = """\
glop_scan_kernel_x:                     ; @glop_scan_kernel_x
	s_load_dwordx2 s[0:1], s[4:5], 0x0
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
	ds_add_rtn_u32 v90, v15, v102
	s_waitcnt lgkmcnt(0)
	ds_add_u64 v14, v[54:55]
	v_add_u32_e32 v11, 0x400, v11
	v_cmp_ge_u32_e32 vcc, v11, v10
	s_cbranch_vccz .LBB0_1
.LBB0_2:
	v_readlane_b32 s0, v112, 35
	v_mov_b64_e32 v[10:11], 0
	s_barrier
	ds_read_b64 v[4:5], v37 offset:128
	s_endpgm
.Lfunc_end0:
"""


def test_flags_a_barrier_reached_with_lds_operations_in_flight(tmp_path):
    got = _check(UNWAITED, tmp_path)
    assert list(got) == ["glop_scan_kernel_x"]
    (problem,) = got["glop_scan_kernel_x"]
    assert problem.startswith("s_barrier at body line") and problem.endswith("without a preceding lgkmcnt(0) wait")


def test_accepts_a_barrier_after_an_explicit_lds_wait(tmp_path):
    fixed = UNWAITED.replace("\ts_barrier\n", "\ts_waitcnt lgkmcnt(0)\n\ts_barrier\n")
    assert _check(fixed, tmp_path) == {}
    # A DS instruction between the wait and the barrier is in flight again.
    late = UNWAITED.replace("\ts_barrier\n", "\ts_waitcnt lgkmcnt(0)\n\tds_write_b32 v65, v37\n\ts_barrier\n")
    assert list(_check(late, tmp_path)) == ["glop_scan_kernel_x"]
