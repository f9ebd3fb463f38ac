"""The mesh builder's host logic on the CPU: tiles, LDS record positions,
tile-local CSR and shared-node partials, checked by a small C++ harness that
compiles the builder's translation unit without any device code
(tests/host/tiles_check.cpp).  Also checks that the bank-aware record
positions lower the modelled gather cycles against the sorted node order."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "tiles_check.cpp")


def _compile(tmp_path_factory, name, defines=()):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("host") / name)
    cmd = [hipcc, "-O1", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-w", "-I/opt/rocm/include",
           *defines, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2602_17002_amd", "csrc"), SRC, "-o", exe, "-L/opt/rocm/lib",
           "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return _compile(tmp_path_factory, "tiles_check")


def _run_raw(harness, tmp_path, X, blocks, flags=0):
    path = tmp_path / "mesh.txt"
    with open(path, "w") as fh:
        fh.write(f"{X.shape[1]} {len(blocks)} {flags}\n")
        fh.write(" ".join(repr(float(v)) for v in X.ravel()) + "\n")
        for b in blocks:
            fh.write(f"{b.elem} {b.law} {int(b.damped)} {getattr(b, 'tile_elems', 0) or 0} {b.conn.shape[0]}\n")
            fh.write(" ".join(str(int(v)) for v in b.conn.ravel()) + "\n")
    env = dict(os.environ, LD_LIBRARY_PATH="/opt/rocm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""),
               ASAN_OPTIONS="detect_leaks=1")
    return subprocess.run([harness, str(path)], capture_output=True, text=True, env=env, timeout=120)


def run(harness, tmp_path, X, blocks, flags=0):
    r = _run_raw(harness, tmp_path, X, blocks, flags)
    out = r.stdout.strip().splitlines()
    assert r.returncode == 0 and out and out[-1].startswith("OK"), (r.stdout[-2000:], r.stderr[-2000:])
    return {k: int(v) for k, v in re.findall(r"(\w+) (\d+)", out[-1])}


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_single_body_tiles(harness, tmp_path, tile):
    X, conn = synth.box_t10(12, 9, 5, size=(0.12, 0.09, 0.05))
    b = synth.Block(synth.T10, synth.NH, conn, np.array([1.7e6, 0, 1.7e7, 1e4, 0]), damped=True)
    b.tile_elems = tile
    s = run(harness, tmp_path, X, [b])
    assert s["tiles"] >= conn.shape[0] // tile
    assert s["gather_cycles_placed"] < 0.8 * s["gather_cycles_sorted"]


@pytest.mark.parametrize("tile", [64, 128])
def test_q27_body_tiles(harness, tmp_path, tile):
    """Q27 tiles hold about 11 nodes per element: at most 12 per thread, and
    the LDS of two 64-element tiles per compute unit; every check of the
    harness (CSR lists, partials, record positions) holds for 27 nodes."""
    X, conn = synth.box_q27(9, 8, 7, size=(0.09, 0.08, 0.07))
    b = synth.Block(synth.Q27, synth.NH, conn, np.array([1.7e6, 0, 1.7e7, 1e4, 0]), damped=True)
    b.tile_elems = tile
    s = run(harness, tmp_path, X, [b])
    assert s["tiles"] >= conn.shape[0] // tile


@pytest.mark.parametrize("tile", [64, 256])
def test_node_in_every_element(harness, tmp_path, tile):
    """One node in all 700 elements (a fan of T10 around it): in every tile
    its slot group is the tile's whole first column of entries and spans
    several threads' chunks (the chunked reduction's long case), and it is
    shared by every tile (one partial per tile)."""
    X, conn = synth.fan_t10(700, 0.02, np.random.default_rng(3))
    b = synth.Block(synth.T10, synth.NH, conn, np.array([1.7e6, 0, 1.7e7, 1e4, 0]), damped=True)
    b.tile_elems = tile
    s = run(harness, tmp_path, X, [b])
    assert s["tiles"] >= 700 // 66 and s["shared"] == 1 and s["partials"] == s["tiles"]


def test_multibody_mixed_blocks_and_keep_order(harness, tmp_path):
    p = synth.config_multibody(6, 150, 2500, seed=21)
    for flags in (0, 4):   # default order, TLFEA_KEEP_ORDER
        s = run(harness, tmp_path, p.X, p.blocks, flags)
        assert s["tiles"] >= len(p.blocks)


def test_shared_nodes_between_blocks(harness, tmp_path):
    # two blocks of one body (T10 halves sharing the middle plane) and a node
    # that no element touches
    X, conn = synth.box_t10(6, 4, 3, size=(0.06, 0.04, 0.03))
    half = conn.shape[0] // 2
    th = np.array([5.8e6, 3.8e6, 0, 0, 0])
    b0 = synth.Block(synth.T10, synth.SVK, conn[:half].copy(), th)
    b1 = synth.Block(synth.T10, synth.NH, conn[half:].copy(), np.array([1.7e6, 0, 1.7e7, 0, 0]))
    X2 = np.concatenate([X, np.full((3, 1), 5.0)], axis=1)
    s = run(harness, tmp_path, X2, [b0, b1])
    # the listed nodes are the shared ones plus the untouched one (no partials)
    assert s["shared"] > 1 and s["partials"] >= 2 * (s["shared"] - 1)


def test_offset_limit_rejects_oversized_mesh(tmp_path_factory, tmp_path):
    # The tile lists use 32-bit offsets (about 200 million T10 elements per
    # mesh).  A harness built with the limit lowered to 3000 entries shows
    # that a mesh above it is refused with UNSUPPORTED instead of wrapping,
    # and that one below it still builds.
    exe = _compile(tmp_path_factory, "tiles_check_limit", ["-DTLFEA_OFFSET_LIMIT=3000"])
    X, conn = synth.box_t10(2, 2, 2, size=(0.02, 0.02, 0.02))      # 48 elements: one 64-element tile
    th = np.array([1.7e6, 0, 1.7e7, 0, 0])
    small = synth.Block(synth.T10, synth.NH, conn, th)
    small.tile_elems = 64
    s = run(exe, tmp_path, X, [small])
    assert s["tiles"] >= 1
    X2, conn2 = synth.box_t10(6, 4, 3, size=(0.06, 0.04, 0.03))    # 432 elements, 4320 node slots
    big = synth.Block(synth.T10, synth.NH, conn2, th)
    big.tile_elems = 64
    r = _run_raw(exe, tmp_path, X2, [big])
    assert "FAIL build_tiles" in r.stdout and "32-bit offset limit" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])


def test_builder_clean_under_address_and_ub_sanitizers(tmp_path_factory, tmp_path):
    # The mesh builder (tiling, lane order, record positions, tile CSR,
    # shared-node partials) compiled for the host alone with GCC's address
    # and undefined-behaviour sanitizers, leak checks on, over T10 tiles of
    # every size, a multibody mesh in both orders and an H8 block.
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "tiles_check_asan")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-w", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2602_17002_amd", "csrc"), SRC, "-o", exe, "-L/opt/rocm/lib", "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    X, conn = synth.box_t10(8, 6, 4, size=(0.08, 0.06, 0.04))
    cases = []
    for te in (64, 128, 192, 256):
        b = synth.Block(synth.T10, synth.NH, conn, np.array([1.7e6, 0, 1.7e7, 1e4, 0]), damped=True)
        b.tile_elems = te
        cases.append((X, [b], 0))
    p = synth.config_multibody(6, 150, 2000, seed=22)
    cases += [(p.X, p.blocks, 0), (p.X, p.blocks, 4)]
    Xh, ch = synth.box_h8(8, 6, 5)
    cases.append((Xh, [synth.Block(synth.H8, synth.MR, ch, np.array([1.2e6, 0.45e6, 1.7e7, 0, 0]))], 0))
    for X_, blocks, flags in cases:
        r = _run_raw(exe, tmp_path, X_, blocks, flags)
        assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-3000:]
        assert r.stdout.strip().splitlines()[-1].startswith("OK"), r.stdout[-1000:]
