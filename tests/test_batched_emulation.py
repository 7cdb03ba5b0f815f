"""CPU emulation of the batched persistent kernel (csrc/batched.hip).

The kernel source is compiled for the host with g++ against a stand-in of the
HIP runtime (tests/emu/hip/hip_runtime.h: a workgroup is 512 host threads,
__syncthreads a barrier, wave collectives exchange through slot arrays).  The
test rewrites a copy of the source so that every LDS array of the workgroup
is bounds checked, builds it with AddressSanitizer and UBSan, gives every
workgroup's key and grade scratch a poisoned tail (tests/emu/batched_emu_main.cpp),
and runs two workgroups on clouds that cover the kernel's edge cases: n = 0,
1 and 2, all distances zero, heavy ties, the largest fused cloud (n = 512),
wide int16 coordinates, with the built-in chunk multipliers, with 1 (many
chunks per cloud) and with 1000 (every edge in the first chunk: the most
scratch a cloud uses), and with 1024-thread workgroups sorting on 5-bit
digits.  Every barcode must equal the oracle's, and the run must end (a
loop that does not end fails the test by its time limit).  CPU only."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_02527_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")

CHECKED = '''
template <typename T, int N>
struct Chk {
  T v[N];
  T& operator[](int64_t k) {
    if (k < 0 || k >= N) {
      fprintf(stderr, "LDS index %lld outside [0, %d)\\n", (long long)k, N);
      abort();
    }
    return v[k];
  }
  const T& operator[](int64_t k) const { return const_cast<Chk*>(this)->operator[](k); }
  operator T*() { return v; }
};
'''


def checked_source() -> str:
    """batched.hip with bounds-checked LDS arrays and the dynamic LDS taken
    from the emulated workgroup."""
    src = open(os.path.join(CSRC, "batched.hip")).read()
    a = src.index("struct Shared {")
    b = src.index("};", a)
    body = src[a:b]
    out = []
    for line in body.splitlines():
        m = re.match(r"^(\s*)(u?int\d+_t) (.*\[.*\]);\s*$", line)
        if not m:
            out.append(line)
            continue
        ind, ty, decls = m.groups()
        for dcl in decls.split(","):
            dm = re.match(r"\s*(\w+)((?:\[[^\]]+\])+)\s*$", dcl)
            assert dm, dcl
            name, dims = dm.group(1), re.findall(r"\[([^\]]+)\]", dm.group(2))
            t = ty
            for dim in reversed(dims):
                t = "Chk<%s, %s>" % (t, dim)
            out.append("%s%s %s;" % (ind, t, name))
    src = src[:a] + "\n".join(out) + src[b:]
    head = "template <int kWaves>\nstruct Shared {"
    assert head in src
    src = src.replace(head, CHECKED + head, 1)
    old = "extern __shared__ __attribute__((aligned(16))) char smem[];"
    assert old in src
    src = src.replace(old, "char* smem = emu_block_smem();")
    return src


def _clouds():
    rng = np.random.default_rng(3)
    return [
        np.array([[5, 5, 5]], np.int16),                          # n = 1
        np.array([[0, 0, 0], [3, 4, 0]], np.int16),                # n = 2
        np.full((40, 3), 7, np.int16),                             # all distances zero
        rng.integers(0, 3, size=(100, 3)).astype(np.int16),        # heavy ties
        rng.integers(-100, 101, size=(512, 3)).astype(np.int16),   # largest fused cloud
        rng.integers(-16000, 16001, size=(65, 3)).astype(np.int16),  # wide int16
        np.zeros((0, 3), np.int16),                                 # empty cloud
        rng.integers(-100, 101, size=(64, 3)).astype(np.int16),
        rng.integers(-100, 101, size=(200, 3)).astype(np.int16),
    ]


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    d = tmp_path_factory.mktemp("emu")
    src = d / "batched_checked.hip.inc"
    src.write_text(checked_source())
    exe = str(d / "batched_emu")
    subprocess.check_call([
        "g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined",
        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-pthread",
        "-Wno-conditionally-supported",
        "-I", EMU, "-I", CSRC, "-I", os.path.join(ROOT, "include"),
        '-DBATCHED_SOURCE="%s"' % str(src),
        os.path.join(EMU, "batched_emu_main.cpp"), "-o", exe])
    return exe, d


def _run(emulator, clouds, chunk_mult, blocks=2, digit_bits=8, threads=512):
    exe, d = emulator
    offsets = np.zeros(len(clouds) + 1, np.int64)
    offsets[1:] = np.cumsum([c.shape[0] for c in clouds])
    pts = np.ascontiguousarray(np.concatenate(clouds, axis=0))
    inp, outp = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        np.array([len(clouds), pts.shape[1], pts.dtype.itemsize, blocks, *chunk_mult,
                  digit_bits, threads], np.int64).tofile(f)
        offsets.tofile(f)
        pts.tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([exe, str(inp), str(outp)], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = np.fromfile(outp, np.uint32)
    rows = int(offsets[-1])
    bars = raw[:2 * rows].reshape(rows, 2)
    errs = raw[2 * rows:].view(np.int32)
    return bars, errs, offsets, pts


@pytest.mark.slow
@pytest.mark.parametrize("chunk_mult,digit_bits,threads", [
    ((6, 6, 8, 48), 8, 512), ((1, 1, 1, 1), 8, 512), ((1000, 1000, 1000, 1000), 8, 512),
    ((1, 1, 1, 1), 5, 1024)])
def test_fused_kernel_edge_cases_on_cpu(emulator, chunk_mult, digit_bits, threads):
    clouds = _clouds()
    bars, errs, offsets, pts = _run(emulator, clouds, chunk_mult, digit_bits=digit_bits,
                                    threads=threads)
    assert not errs.any(), errs
    for c in range(len(clouds)):
        lo, hi = int(offsets[c]), int(offsets[c + 1])
        if hi == lo:
            continue
        ref = oracle.barcode(pts[lo:hi]).canonical
        assert (bars[lo:hi, 0] == 0).all(), c
        np.testing.assert_array_equal(bars[lo:hi, 1], ref, err_msg="cloud %d" % c)


def test_checked_source_rewrites_every_lds_array():
    src = checked_source()
    body = src[src.index("struct Shared {"):src.index("};", src.index("struct Shared {"))]
    assert "Chk<" in body
    assert not re.search(r"^\s*u?int\d+_t \w+\[", body, re.M), body
