"""Host-side logic of the library, checked without a GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serving_arena_allocator(tmp_path):
    """First-fit allocation never overlaps, refuses only when no free run is
    large enough, keeps its accounting, and coalesces back to one block
    (compiled with g++ under AddressSanitizer/UBSan on the host)."""
    exe = tmp_path / "arena_check"
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                           os.path.join(HERE, "arena_check.cpp"), "-o", str(exe)])
    for seed in (1, 2, 3):
        out = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr


def test_result_status_mapping(tmp_path):
    """Status bits raised by the update-step kernels map to the C-ABI statuses
    (input errors before a non-finite result), as read_result and the server
    apply them; compiled on the host from the HIP-free header."""
    exe = tmp_path / "status_check"
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                           os.path.join(HERE, "status_check.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_bench_sphere_image_count(bc):
    """bench.py counts the sphere near set (for its pair totals) exactly as the
    oracle builds it."""
    import math

    import numpy as np

    import bench
    import oracle
    from oracle import hsma as oh
    from paper_1806_04801_amd import workloads as W
    x, q = W.slab_charges(50, 1.0, 2) if bc == 2 else W.uniform_neutral(50, 1.0, 2)
    R = 1.7 * math.sqrt(3) / 2
    cfg = dict(L=1.0, R=R, bc=bc)
    c = oh.normalize(x, 1.0, bc)
    if bc == 2:
        c, q = oh.double_slab(c, q)
    img, _, _ = oracle.sphere_images(oracle.BC_METALLIC if bc == 1 else oracle.BC_PERIODIC, 1.0,
                                     np.concatenate([c, q[:, None]], axis=1), R)
    assert bench.sphere_image_count(x, cfg) == len(img)


def test_bench_traffic_needs_matching_kernel_source(tmp_path, monkeypatch):
    import shutil

    import bench
    csrc = os.path.join(os.path.dirname(HERE), "paper_1806_04801_amd", "csrc")
    (tmp_path / "paper_1806_04801_amd" / "csrc").mkdir(parents=True)
    for name in ("pairs.hip", "sym.hip", "pair_math.h"):
        shutil.copy(os.path.join(csrc, name), tmp_path / "paper_1806_04801_amd" / "csrc" / name)
    prof = tmp_path / "profiles"
    prof.mkdir()
    h_tiles = bench.kernel_source_hash("tiles")
    h_once = bench.kernel_source_hash("pair-once")
    assert h_tiles != h_once
    (prof / "near_f32_w_pmc.md").write_text(
        "- hbm_bytes_per_launch: 123.5\n- kernel_source_sha256_16: %s   (x)\n" % h_tiles)
    (prof / "near_pair_once_f32_w_pmc.md").write_text(
        "- hbm_bytes_per_launch: 77.0\n- kernel_source_sha256_16: %s   (x)\n" % h_once)
    (prof / "near_f32_v_pmc.md").write_text(
        "- hbm_bytes_per_launch: 123.5\n- kernel_source_sha256_16: 0000000000000000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("w", "f32") == 123.5
    assert bench.profiled_traffic("w", "f32", "pair-once") == 77.0
    assert bench.profiled_traffic("v", "f32") is None
    assert bench.profiled_traffic("missing", "f32") is None
    # a summary of one kernel does not serve the other
    (prof / "near_pair_once_f32_v_pmc.md").write_text(
        "- hbm_bytes_per_launch: 5.0\n- kernel_source_sha256_16: %s   (x)\n" % h_tiles)
    assert bench.profiled_traffic("v", "f32", "pair-once") is None
    # a comment does not change the code; an edit to the shared arithmetic
    # invalidates both
    with open(tmp_path / "paper_1806_04801_amd" / "csrc" / "pair_math.h", "a") as f:
        f.write("// a comment\n")
    assert bench.profiled_traffic("w", "f32") == 123.5
    with open(tmp_path / "paper_1806_04801_amd" / "csrc" / "pair_math.h", "a") as f:
        f.write("static int edit_marker;\n")
    assert bench.profiled_traffic("w", "f32") is None
    assert bench.profiled_traffic("w", "f32", "pair-once") is None


def test_own_image_constants_match_lattice_sums():
    """The own-image constants that the near-sum kernels leave to the finalize
    stage equal the lattice sums they stand for: the potential of the 26
    images k != 0 of the periodic 3x3x3 block of a unit charge at the origin
    (box side 1), and its split over the nine columns (k_x, k_y), which the
    single-precision kernels subtract as float values."""
    import itertools
    import re

    import numpy as np

    src = open(os.path.join(HERE, "..", "paper_1806_04801_amd", "csrc", "hsma_internal.h")).read()

    def const(name):
        m = re.search(r"constexpr (?:float|double) %s = ([0-9.]+)f?;" % name, src)
        assert m, name
        return float(m.group(1))

    total = const("OWN_IMAGES_PERIODIC")
    cols = {}
    for kx, ky in itertools.product((-1, 0, 1), repeat=2):
        cols[(kx, ky)] = sum(1.0 / np.sqrt(kx * kx + ky * ky + kz * kz)
                             for kz in (-1, 0, 1) if (kx, ky, kz) != (0, 0, 0))
    brute = sum(cols.values())
    assert abs(total - brute) <= 1e-15 * brute
    # closed form 6 + 12/sqrt(2) + 8/sqrt(3): faces, edges, corners of the cube
    assert abs(brute - (6 + 12 / np.sqrt(2) + 8 / np.sqrt(3))) <= 1e-14
    centre, edge, corner = const("OWN_COL_CENTRE"), const("OWN_COL_EDGE"), const("OWN_COL_CORNER")
    assert np.float32(centre) == np.float32(cols[(0, 0)])
    assert np.float32(edge) == np.float32(cols[(1, 0)]) == np.float32(cols[(0, -1)])
    assert np.float32(corner) == np.float32(cols[(1, 1)]) == np.float32(cols[(-1, 1)])
    # the nine float constants add up to the total within float rounding
    shift = float(np.float32(centre)) + 4 * float(np.float32(edge)) + 4 * float(np.float32(corner))
    assert abs(shift - total) <= 9 * 2.0 ** -22


def test_header_documents_every_environment_override():
    """Every environment variable that the library reads is named in the
    public header, where its meaning and the values it accepts are stated."""
    import glob
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    names = set()
    for path in glob.glob(os.path.join(root, "paper_1806_04801_amd", "csrc", "*")):
        text = open(path).read()
        # every "HSMA_..." string literal of the sources is a variable name
        names |= set(re.findall(r'"(HSMA_[A-Z0-9_]+)"', text))
    assert {"HSMA_SYM", "HSMA_OVERLAP", "HSMA_TPL_NEAR"} <= names
    header = open(os.path.join(root, "include", "hsma.h")).read()
    missing = sorted(n for n in names if not re.search(r"\b%s\b" % n, header))
    assert not missing, missing


@pytest.mark.parametrize("n,block,bc", [(10, 4, 0), (3000, 1536, 1), (1000, 1000, 0), (77, 20, 2)])
def test_bench_counts_evaluated_near_pairs(n, block, bc):
    """bench.py's roofline charges 20 flops per pair-image the pair-once
    kernel evaluates: each cross-block unordered pair once, every ordered pair
    (self included) inside a diagonal block; counted here by brute force."""
    import bench
    blocks = (n + block - 1) // block
    sched = {"kind": 1, "block": block, "blocks": blocks}
    blk = [i // block for i in range(n)]
    cnt = 0
    for i in range(n if n <= 100 else 0):
        for j in range(n):
            if blk[i] == blk[j]:
                cnt += 1
            elif i < j:
                cnt += 1
    if n > 100:
        sizes = [min(block, n - b * block) for b in range(blocks)]
        cnt = sum(s * s for s in sizes) + sum(sizes[a] * sizes[b] for a in range(blocks)
                                              for b in range(a + 1, blocks))
    imgs = 54 if bc == 2 else 27
    assert bench.near_evaluated_pairs(n, {"bc": bc}, sched) == imgs * cnt
    tiles = bench.near_evaluated_pairs(n, {"bc": bc}, {"kind": 0})
    assert tiles == 27.0 * n * (2 * n if bc == 2 else n)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of hsma_plan_desc and hsma_plan_info_t have the C
    header's size and field offsets (a C program prints them)."""
    import ctypes

    from paper_1806_04801_amd import hsma
    exe = tmp_path / "layout_check"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(HERE, "..", "include"),
                           os.path.join(HERE, "layout_check.c"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout
    types = {"hsma_plan_desc": hsma.PlanDesc, "hsma_plan_info_t": hsma.PlanInfo}
    seen = set()
    for line in out.strip().splitlines():
        name, size, *fields = line.split()
        T = types[name]
        assert ctypes.sizeof(T) == int(size), name
        assert [f for f, _ in T._fields_] == [kv.split("=")[0] for kv in fields], name
        for kv in fields:
            f, off = kv.split("=")
            assert getattr(T, f).offset == int(off), (name, f)
        seen.add(name)
    assert seen == set(types)
