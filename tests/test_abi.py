"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU), and stays independent of the
oracle."""
import ctypes as ct
import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "rotvote.h"
PROBE_HEADER = ROOT / "include" / "rotvote_probe.h"
LIB = ROOT / "paper_2506_11547_amd" / "librotvote.so"
PROBE = ROOT / "paper_2506_11547_amd" / "librotvote_probe.so"


def declared():
    text = HEADER.read_text()
    return sorted(set(re.findall(r"\b(rot_vote_\w+)\s*\(", text)))


def dynamic_symbols(lib: Path):
    out = subprocess.run(["nm", "-D", "--defined-only", str(lib)], capture_output=True,
                         text=True, check=True).stdout
    return {ln.split()[-1] for ln in out.splitlines() if ln.strip()}


@pytest.fixture(scope="module")
def lib_path():
    if not LIB.exists():
        pytest.fail("librotvote.so is not built (run __graft_entry__.build())")
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for need in ("rot_vote_create", "rot_vote_solve", "rot_vote_destroy", "rot_vote_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(lib_path):
    syms = dynamic_symbols(lib_path)
    missing = [n for n in declared() if n not in syms]
    assert not missing, missing
    # nothing but the C-ABI is exported
    extra = [s for s in syms if s.startswith("rot_vote") and s not in declared()]
    assert not extra, extra
    lib = ct.CDLL(str(lib_path))
    for n in declared():
        assert getattr(lib, n) is not None


def test_binding_names_match_header():
    from paper_2506_11547_amd import rotvote
    assert sorted(rotvote.EXPORTS) == declared()


def test_product_library_does_not_reference_the_oracle(lib_path):
    out = subprocess.run(["nm", "-D", str(lib_path)], capture_output=True, text=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["readelf", "-d", str(lib_path)], capture_output=True, text=True).stdout
    assert "liborc" not in ldd
    for src in (ROOT / "paper_2506_11547_amd").rglob("*"):
        if src.suffix in (".py", ".hip", ".cpp", ".h"):
            text = src.read_text()
            assert "import oracle" not in text and "from oracle" not in text, src
            assert "rotvote_oracle" not in text, src


def test_probe_library_exports_its_header(lib_path):
    declared_probe = sorted(set(re.findall(r"\b(rvp_\w+)\s*\(", PROBE_HEADER.read_text())))
    assert len(declared_probe) == 12, declared_probe
    syms = dynamic_symbols(PROBE)
    assert [n for n in declared_probe if n not in syms] == []
    assert [s for s in syms if s.startswith("rvp_") and s not in declared_probe] == []


def test_default_config_and_create_without_gpu(lib_path):
    from paper_2506_11547_amd.rotvote import RvConfig
    lib = ct.CDLL(str(lib_path))
    cfg = RvConfig()
    lib.rot_vote_default_config(ct.byref(cfg))
    assert cfg.max_grid == 256 and cfg.topk == 16 and cfg.samples_per_circle == 0
    lib.rot_vote_create.argtypes = [ct.POINTER(ct.c_void_p), ct.POINTER(RvConfig)]
    lib.rot_vote_last_error.restype = ct.c_char_p
    lib.rot_vote_last_error.argtypes = [ct.c_void_p]
    bad = RvConfig()
    lib.rot_vote_default_config(ct.byref(bad))
    bad.topk = 65
    h = ct.c_void_p()
    assert lib.rot_vote_create(ct.byref(h), ct.byref(bad)) == -1
    assert b"topk" in lib.rot_vote_last_error(None)
    assert not h.value
    cfg_sz = ct.sizeof(RvConfig)
    assert cfg_sz == 64, cfg_sz  # rv_config: 4 + 4 pad + 8 + 8 + 4*4 + 4 + 4 + 4 + 4 + 8
    from paper_2506_11547_amd.rotvote import RigidParams, RigidResult
    assert ct.sizeof(RigidParams) == 32 and ct.sizeof(RigidResult) == 64
    for field, value, word in (("max_pairs", 1 << 21, b"max_pairs"), ("max_pairs", -1, b"max_pairs"),
                               ("reserved", 1, b"reserved")):
        bad = RvConfig()
        lib.rot_vote_default_config(ct.byref(bad))
        assert bad.max_pairs == 0
        setattr(bad, field, value)
        assert lib.rot_vote_create(ct.byref(h), ct.byref(bad)) == -1, field
        assert word in lib.rot_vote_last_error(None)
        assert not h.value
    bad = RvConfig()
    lib.rot_vote_default_config(ct.byref(bad))
    assert bad.max_batch == 0
    bad.max_batch = 4
    bad.vote_strategy = 1  # global: batches need the brick strategy
    assert lib.rot_vote_create(ct.byref(h), ct.byref(bad)) == -4
    assert b"batch" in lib.rot_vote_last_error(None)
    bad.max_batch = -1
    bad.vote_strategy = 0
    assert lib.rot_vote_create(ct.byref(h), ct.byref(bad)) == -1
    assert not h.value


def test_server_config_checks_without_gpu(lib_path):
    from paper_2506_11547_amd.rotvote import ServerConfig
    lib = ct.CDLL(str(lib_path))
    lib.rot_vote_server_create.argtypes = [ct.POINTER(ct.c_void_p), ct.POINTER(ServerConfig)]
    lib.rot_vote_server_last_error.restype = ct.c_char_p
    lib.rot_vote_server_last_error.argtypes = [ct.c_void_p]
    assert ct.sizeof(ServerConfig) == 72  # 4 4 8 4 4 4 4 8 8 8 16
    from paper_2506_11547_amd.rotvote import Reply, Request
    assert ct.sizeof(Request) == 56  # 8 8 8 4 4 8 4 4 8
    assert ct.sizeof(Reply) == 72    # 16 8 4 4 4 4 8 8 8 8
    cfg = ServerConfig()
    lib.rot_vote_server_default_config(ct.byref(cfg))
    assert cfg.workers == 4 and cfg.max_batch == 64 and cfg.hbm_budget == 0
    h = ct.c_void_p()
    for field, value in (("workers", 0), ("workers", 65), ("max_queue", 0), ("max_n", 0)):
        bad = ServerConfig()
        lib.rot_vote_server_default_config(ct.byref(bad))
        setattr(bad, field, value)
        assert lib.rot_vote_server_create(ct.byref(h), ct.byref(bad)) == -1, field
        assert lib.rot_vote_server_last_error(None)
    bad = ServerConfig()
    lib.rot_vote_server_default_config(ct.byref(bad))
    bad.reserved[2] = 1
    assert lib.rot_vote_server_create(ct.byref(h), ct.byref(bad)) == -1
    assert not h.value
