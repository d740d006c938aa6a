"""Host-side checks of the benchmark's bookkeeping (no GPU needed): the stored
HBM traffic of the mixed-precision solve is reported only for the kernel
sources and solve tolerances its counter runs were taken with."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_traffic_tied_to_sources_and_tolerances():
    B = _bench()
    T = B.SOLVE_TRAFFIC
    got = B.solve_traffic_bytes(T["tol"], T["tol_inner"])
    if T["sha256"] is None or B.sources_sha256(T["sources"]) != T["sha256"]:
        # counter runs older than the kernel sources: no traffic is reported
        assert got is None
        return
    want = 1024.0 * (T["fetch_kib"] * T["fetch_factor"] + T["write_kib"] * T["write_factor"])
    assert got == want and got > 0
    assert B.solve_traffic_bytes(T["tol"], T["tol_inner"] * 10) is None
    assert B.solve_traffic_bytes(T["tol"] * 10, T["tol_inner"]) is None


def test_default_tolerances_match_measured_traffic():
    B = _bench()
    ap_defaults = {}
    src = open(os.path.join(ROOT, "bench.py")).read()
    for key in ("--tol", "--tol-inner"):
        i = src.index(f'ap.add_argument("{key}"')
        seg = src[i:src.index(")", i)]
        ap_defaults[key] = float(seg.split("default=")[1].split(",")[0])
    assert ap_defaults["--tol"] == B.SOLVE_TRAFFIC["tol"]
    assert ap_defaults["--tol-inner"] == B.SOLVE_TRAFFIC["tol_inner"]
