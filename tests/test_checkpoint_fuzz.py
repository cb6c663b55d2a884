"""The checkpoint reader against crafted files, under AddressSanitizer and
UndefinedBehaviorSanitizer on the host (CPU, no device): the library is built
with the sanitizers on its host code only, and llr_checkpoint_info reads a
well-formed file and about a thousand mutations of it whose CRC has been
recomputed, so that the parser, not the checksum, has to refuse them: random
bytes in the header, every 32- and 64-bit field of the header and of the
section table set to extreme values, and the file cut inside and between
sections.  Every file must be accepted or refused without a memory error or
an undefined operation, and the library's verdict on each file must be that
of a validator of the documented layout written here, independently of the
library: accepted exactly when the header holds values llr_add_lattice and
llr_set_params accept and the section table covers the rest of the file with
every section present once at the size the header implies."""
import os
import struct
import subprocess
import zlib
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from tests.test_checkpoint_file import LATS, PRM, _file, full_sections, section_sizes

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1509_08391_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang"
SOURCES = ("llr_capi.hip", "llr_recon.hip", "llr_mlp.hip", "llr_sweep.hip")
# sanitizers on the host code only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _valid(data):
    """The documented checkpoint layout, checked field by field."""
    if len(data) < 16 or data[:8] != b"LLRCKPT1":
        return False
    if zlib.crc32(data[:-4]) & 0xFFFFFFFF != struct.unpack_from("<I", data, len(data) - 4)[0]:
        return False
    end, off = len(data) - 4, 8

    def take(fmt):
        nonlocal off
        k = struct.calcsize(fmt)
        if k > end - off:
            raise ValueError
        v = struct.unpack_from(fmt, data, off)
        off += k
        return v

    try:
        ver, prec, nl = take("<III")
        if ver != 2 or prec not in (0, 1) or not 1 <= nl <= 8:
            return False
        lats = []
        for _ in range(nl):
            L, n, dE = take("<iid")
            if not (2 <= L <= 32 and L % 2 == 0 and 1 <= n <= 4096 and dE > 0):
                return False
            E = take(f"<{n}d")
            six_v = 6.0 * L ** 4
            for k, e in enumerate(E):
                if not np.isfinite(e) or (k and not e > E[k - 1]) or e < -six_v or e + dE > six_v:
                    return False
            lats.append((L, n))
        n_th, n_a, n_rm, _, _, overlap, rec, eps, cap = take("<iiiQidid" + "i")
        if n_a < 1 or n_th < 0 or n_rm < 0 or rec < 1 or cap < 0 or not eps >= 0 or not overlap >= 0:
            return False
        secs = {}
        while off < end:
            tag, nbytes = take("<IQ")
            if nbytes > end - off or not 1 <= tag <= 24 or tag in secs:
                return False
            secs[tag] = nbytes
            off += nbytes
    except ValueError:
        return False
    want = dict(section_sizes([(L, [0.0] * n, 1.0) for L, n in lats], n_rm, precision=prec))
    n_ch = sum(n for _, n in lats)
    if 15 not in secs or secs[15] not in (0, 8 * (n_rm + 1) * n_ch):
        return False
    return all(secs.get(t) == k for t, k in want.items() if t != 15)


def _with_crc(body):
    return body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF)


def _layout(lats):
    """Byte offsets of the header fields and of every section's tag and size."""
    off = 8 + 12
    fields = [(8, 4), (12, 4), (16, 4)]
    for _, E, _ in lats:
        fields += [(off, 4), (off + 4, 4), (off + 8, 8)]
        off += 16 + 8 * len(E)
    for size in (4, 4, 4, 8, 4, 8, 4, 8, 4):              # the parameters
        fields.append((off, size))
        off += size
    return fields, off


def _mutations(good, secs, rng):
    body = good[:-4]
    fields, first = _layout(LATS)
    sec_heads, off = [], first
    for _, data in secs:
        sec_heads += [(off, 4), (off + 4, 8)]
        off += 12 + len(data)
    assert off == len(body)
    out = [good]
    for _ in range(200):                                   # random bytes in the header
        b = bytearray(body)
        for _ in range(int(rng.integers(1, 4))):
            b[int(rng.integers(0, first))] = int(rng.integers(0, 256))
        out.append(_with_crc(bytes(b)))
    extremes = {4: [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF],
                8: [0, 1, 0x7FF0000000000000, 0x7FFFFFFFFFFFFFFF, 0x8000000000000000, 0xFFFFFFFFFFFFFFFF]}
    for at, size in fields + sec_heads:                    # every field at its extremes
        for v in extremes[size]:
            b = bytearray(body)
            b[at:at + size] = v.to_bytes(size, "little")
            out.append(_with_crc(bytes(b)))
    for at, _ in sec_heads[::2]:                           # cut at, and just inside, every section
        out.append(_with_crc(body[:at]))
        out.append(_with_crc(body[:at + 7]))
        out.append(_with_crc(body[:at + 13]))
    for cut in rng.integers(8, len(body), 50):             # cut anywhere
        out.append(_with_crc(body[:int(cut)]))
    return out


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr[-3000:]


def test_checkpoint_reader_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc or clang not available")
    objs = [str(tmp_path / s.replace(".hip", ".o")) for s in SOURCES]
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        list(ex.map(_run, [[HIPCC, *DEVICE, "-O1", "-g", "-std=c++17", "-fPIC", *HOST_SAN, "-c",
                            os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]))
    lib = str(tmp_path / "libllr_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, *objs, "-o", lib])
    # the driver is C, built by the same clang so that one sanitizer runtime serves both
    exe = str(tmp_path / "ckpt_fuzz")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(HERE, "csrc", "ckpt_fuzz_driver.c"), lib, f"-Wl,-rpath,{tmp_path}", "-o", exe])

    secs = full_sections(LATS, PRM[2])
    good = _file(LATS, PRM, sections=secs)
    files = []
    for i, data in enumerate(_mutations(good, secs, np.random.default_rng(1509))):
        p = tmp_path / f"m{i}.ckpt"
        p.write_bytes(data)
        files.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    got = r.stdout.strip()
    assert len(got) == len(files)
    want = "".join("A" if _valid(open(f, "rb").read()) else "R" for f in files)
    assert want[0] == "A"                                  # the well-formed file
    assert 10 <= want.count("A") <= len(files) - 100        # both verdicts are exercised
    wrong = [i for i in range(len(files)) if got[i] != want[i]]
    assert not wrong, f"{len(wrong)} verdicts differ, first file m{wrong[0]}: library {got[wrong[0]]}"
