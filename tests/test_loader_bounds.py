"""The digit pass's tile loads stay inside the caller's arrays.  CPU only.

A tile of `len` records starting at record `start` is loaded through one raw buffer resource
whose base is the tile's first record and whose size is exactly len * sizeof(T) bytes.  The
hardware range check of a raw (unswizzled) buffer access covers the vector offset plus the
instruction's immediate offset; the scalar offset is added to the address outside that check.
So a load is provably inside [start, start + len) when

  1. every buffer load of the built kernels takes its scalar offset from the literal 0 (checked
     on the device code of the built libqsd.so), and
  2. under the loader's addressing (lane offset in the vector register, per-item constants of
     at most 4095 bytes in the immediate field, larger multiples of 4096 added to the vector
     register), every access that passes the check lies inside the tile, and every record the
     kernel keeps (index < len) is one that passes (checked by enumerating every wave, lane,
     item and partial-tile length).
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from conftest import ROOT

LIB = os.path.join(ROOT, "paper_2005_10427_amd", "libqsd.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
BLOCK = 256


def _device_disassembly():
    if not os.path.exists(LIB):
        pytest.fail("libqsd.so is not built (run __graft_entry__.build())")
    if not os.path.exists(OBJDUMP):
        pytest.skip("llvm-objdump not available")
    with tempfile.TemporaryDirectory(prefix="qsd_dis_") as tmp:
        lib = os.path.join(tmp, "libqsd.so")
        shutil.copy(LIB, lib)
        subprocess.run([OBJDUMP, "--offloading", lib], cwd=tmp, check=True, capture_output=True)
        texts = []
        for fn in sorted(os.listdir(tmp)):
            if "amdgcn" in fn and "gfx950" in fn:
                res = subprocess.run([OBJDUMP, "-d", os.path.join(tmp, fn)], check=True,
                                     capture_output=True, text=True)
                texts.append(res.stdout)
    assert texts, "no gfx950 code object in libqsd.so"
    return "\n".join(texts)


BUF = re.compile(r"^\s*(buffer_(?:load|store)\w*)\s+([^/]*?)\s*(?://|$)")


def test_buffer_accesses_have_no_scalar_offset():
    dis = _device_disassembly()
    n = 0
    for line in dis.splitlines():
        m = BUF.match(line)
        if not m:
            continue
        n += 1
        ops = [o.strip() for o in m.group(2).split(",")]
        # vdata, vaddr, srsrc, soffset [offen] [offset:imm]
        assert len(ops) >= 4, line
        tail = ops[3].split()
        assert tail[0] == "0", f"scalar offset in a buffer access: {line.strip()}"
        assert "offen" in tail, f"buffer access without a vector offset: {line.strip()}"
        imm = [int(t.split(":")[1]) for t in tail if t.startswith("offset:")]
        assert all(0 <= x <= 4095 for x in imm), line
    assert n > 0, "no buffer accesses found"


def _loader_offsets(wave, lane, items, size):
    """(vector, immediate) byte offsets of each item as the loader issues them."""
    wb = wave * 64 * items + lane
    out = []
    for i in range(items):
        const = i * 64 * size
        over = const & ~4095  # the part that does not fit the 12-bit immediate
        out.append((wb * size + over, const - over))
    return wb, out


@pytest.mark.parametrize("size,items", [(4, 16), (8, 16), (4, 8), (8, 8)])
def test_every_load_of_a_partial_tile_stays_inside(size, items):
    tile = BLOCK * items
    lengths = sorted(set(list(range(1, 130)) + list(range(tile - 130, tile + 1, 1)) +
                         list(range(1, tile + 1, 61))))
    for length in lengths:
        limit = length * size  # num_records of the resource, in bytes
        kept = set()
        for wave in range(BLOCK // 64):
            for lane in range(64):
                wb, offs = _loader_offsets(wave, lane, items, size)
                for i, (v, imm) in enumerate(offs):
                    off = v + imm
                    assert off == (wb + 64 * i) * size
                    passes = off < limit  # raw buffer: offset = vector + immediate
                    if passes:
                        # the whole access is inside the tile's bytes
                        assert off + size <= limit
                    rec = wb + 64 * i
                    if rec < length:  # the kernel keeps this item: it must have been loaded
                        assert passes
                        kept.add(rec)
                    else:  # masked by index; the load returned 0 without an access
                        assert not passes
        assert kept == set(range(length))
