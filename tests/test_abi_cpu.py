"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/dns.h declares, and rejects invalid arguments before
touching the device."""
import ctypes

import pytest

import paper_1602_03638_amd as dns
from paper_1602_03638_amd import binding


@pytest.fixture(scope="module")
def lib():
    return dns.load_library()


def test_exports_every_declared_function(lib):
    names = dns.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_covers_status_codes(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.dns_strerror(code)
    assert lib.dns_strerror(12345) == b"unknown status"


def test_default_opts(lib):
    o = dns.default_opts()
    assert (o.dealias, o.diag_every, o.history_cap, o.use_graph, o.autotune, o.fuse, o.integrator,
            o.mfma_dft) == (0, 0, 4096, 1, 0, 1, 0, 0)


def test_state_bytes(lib):
    # 15 half-spectrum fields of N*N*(N/2+1) complex values, each iz row and
    # ix plane padded by 128 bytes (+ a small twiddle table)
    b = dns.state_bytes(512, dns.DNS_FP64)
    field = 512 * 512 * 257 * 16
    padded = (512 * (512 * (256 + 8) + 8) + 512 * 512) * 16
    assert 15 * field < 15 * padded <= b < 15 * padded + (1 << 20)
    assert dns.state_bytes(512, dns.DNS_FP32) < b
    assert dns.state_bytes(500, dns.DNS_FP64) == 0
    assert dns.state_bytes(2048, dns.DNS_FP64) == 0
    assert dns.state_bytes(64, 7) == 0


@pytest.mark.parametrize("args", [
    (6, 0.01, 0.01, 0),        # N not a power of two >= 8
    (12, 0.01, 0.01, 0),
    (2048, 0.01, 0.01, 0),     # N too large
    (32, -1.0, 0.01, 0),       # negative viscosity
    (32, float("nan"), 0.01, 0),
    (32, 0.01, 0.0, 0),        # non-positive dt
    (32, 0.01, float("inf"), 0),
    (32, 0.01, 0.01, 2),       # bad dtype
])
def test_create_rejects_invalid_arguments(lib, args):
    h = ctypes.c_void_p(123)
    st = lib.dns_create(*args, ctypes.byref(h))
    assert st == dns.DNS_E_INVAL
    assert not h.value


def test_create_rejects_bad_opts(lib):
    o = dns.default_opts()
    o.dealias = 5
    h = ctypes.c_void_p()
    assert lib.dns_create_ex(32, 0.01, 0.01, 0, ctypes.byref(o), None, ctypes.byref(h)) == dns.DNS_E_INVAL
    o = dns.default_opts()
    o.diag_every = -1
    assert lib.dns_create_ex(32, 0.01, 0.01, 0, ctypes.byref(o), None, ctypes.byref(h)) == dns.DNS_E_INVAL


def test_null_handles_are_rejected(lib):
    assert lib.dns_create(32, 0.01, 0.01, 0, None) == dns.DNS_E_INVAL
    assert lib.dns_destroy(None) == dns.DNS_OK
    assert lib.dns_step(None, 1) == dns.DNS_E_INVAL
    assert lib.dns_set_velocity(None, None) == dns.DNS_E_INVAL
    assert lib.dns_energy(None, None) == dns.DNS_E_INVAL
    assert lib.dns_synchronize(None) == dns.DNS_E_INVAL
    assert lib.dns_last_error(None) == b""


def test_binding_signatures_cover_header():
    lib = dns.load_library()
    for n in dns.header_functions():
        assert getattr(lib, n).argtypes is not None or n == "dns_default_opts", n


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="build"):
        binding.load_library(str(tmp_path / "nope.so"))


def test_plan_cache_starts_empty_and_clears(lib):
    # no context has been tuned in this CPU-only process
    dns.plan_cache_clear()
    assert dns.plan_cache_entries() == 0


def test_workspace_bytes_and_validation(lib):
    b = dns.workspace_bytes(512, dns.DNS_FP64)
    assert b == dns.state_bytes(512, dns.DNS_FP64) > 0
    assert dns.workspace_bytes(512, dns.DNS_FP32) < b
    # a longer history needs more room; invalid options need none
    assert dns.workspace_bytes(64, dns.DNS_FP64, history_cap=100000) > dns.workspace_bytes(64, dns.DNS_FP64)
    assert dns.workspace_bytes(64, dns.DNS_FP64, mfma_dft=1) == 0       # FP64 has no matrix-core stage
    assert dns.workspace_bytes(64, dns.DNS_FP32, mfma_dft=1) > dns.workspace_bytes(64, dns.DNS_FP32)
    assert dns.workspace_bytes(48, dns.DNS_FP64) == 0
    # a null workspace is rejected before any device call
    h = ctypes.c_void_p()
    assert lib.dns_create_ws(64, 0.01, 0.01, dns.DNS_FP64, None, None, 1 << 30, None, ctypes.byref(h)) == \
        dns.DNS_E_INVAL


def test_plan_cache_file_round_trip(tmp_path):
    """The tuned-plan cache file (dns_plan_cache_save / _load, no GPU needed):
    plans read from a file are counted, written back as valid JSON with the
    same descriptors, and cleared."""
    import json
    import paper_1602_03638_amd as dns
    lib = dns.load_library()
    lib.dns_plan_cache_clear()
    src = tmp_path / "plans.json"
    src.write_text(
        '{"format": "dns-plan-cache-2", "plans": [\n'
        '{"device": "gfx950|MI355X|256", "N": 512, "dtype": 0, "members": 1, "mode": 0, "variants": '
        '[[8, 0, 0, 1, 0, 0], [8, 0, 8, 1, 0, 0], [4, 0, 0, -1, 0, 8], [8, 0, 8, -1, 0, 0], [8, 0, 0, -1, 0, 0], '
        '[8, 0, 0, 1, 0, 0]]},\n'
        '{"device": "gfx950|MI355X|256", "N": 512, "dtype": 0, "members": 1, "mode": 1, "variants": '
        '[[8, 0, 0, 1, 2, 0], [8, 0, 8, 1, 2, 0], [4, 0, 0, -1, 0, 16], [8, 0, 8, -1, 2, 0], [8, 0, 0, -1, 0, 0], '
        '[8, 0, 0, 1, 2, 0]]},\n'
        '{"device": "gfx950|MI355X|256", "N": 1024, "dtype": 1, "members": 1, "mode": 0, "variants": '
        '[[8, 1, 0, 0, 0, 0], [16, 0, 32, 0, 0, 0], [2, 0, 0, -1, 0, 8], [16, 0, 32, -1, 0, 0], [8, 1, 0, -1, 0, 0], '
        '[8, 1, 0, 0, 0, 0]]},\n'
        # a line of the earlier four-field format and one with an unknown mode are skipped
        '{"device": "gfx950|MI355X|256", "N": 256, "dtype": 0, "members": 1, "variants": '
        '[[8, 0, 0, 1], [8, 0, 8, 1], [4, 0, 0, -1], [8, 0, 8, -1], [8, 0, 0, -1], [8, 0, 0, 1]]},\n'
        '{"device": "gfx950|MI355X|256", "N": 128, "dtype": 0, "members": 1, "mode": 5, "variants": '
        '[[8, 0, 0, 1, 0, 0], [8, 0, 8, 1, 0, 0], [4, 0, 0, -1, 0, 8], [8, 0, 8, -1, 0, 0], [8, 0, 0, -1, 0, 0], '
        '[8, 0, 0, 1, 0, 0]]}\n'
        ']}\n')
    assert dns.plan_cache_load(str(src)) == 3
    assert dns.plan_cache_entries() == 3
    out = tmp_path / "out.json"
    dns.plan_cache_save(str(out))
    rec = json.loads(out.read_text())
    assert rec["format"] == "dns-plan-cache-2" and len(rec["plans"]) == 3
    by_key = {(p["N"], p["mode"]): p for p in rec["plans"]}
    assert by_key[(1024, 0)]["variants"][0] == [8, 1, 0, 0, 0, 0] and by_key[(1024, 0)]["dtype"] == 1
    assert by_key[(512, 0)]["variants"][1] == [8, 0, 8, 1, 0, 0]
    assert by_key[(512, 0)]["device"] == "gfx950|MI355X|256"
    assert by_key[(512, 1)]["variants"][2] == [4, 0, 0, -1, 0, 16] and by_key[(512, 1)]["variants"][0][4] == 2
    with pytest.raises(dns.DnsError):
        dns.plan_cache_load(str(tmp_path / "missing.json"))
    dns.plan_cache_clear()
    assert dns.plan_cache_entries() == 0
