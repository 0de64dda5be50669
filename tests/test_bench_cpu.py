"""Host logic of bench.py that needs no GPU: the hash that ties the HBM traffic counters in
profiles/traffic.json to the library sources they were taken on, and the byte counts the
roofline entry divides by."""
import json

import bench


def test_code_hash_ignores_comments_and_layout():
    src = 'int f(int a) {\n    // sum "x"\n    return a + 1; /* one */\n}\nconst char *s = "a // b";\n'
    same = 'int f(int a)\n{ return a + 1;\n}\n// trailing\nconst char *s = "a // b";'
    other = 'int f(int a) { return a + 2; }\nconst char *s = "a // b";'
    assert bench._code_only(src) == bench._code_only(same)
    assert bench._code_only(src) != bench._code_only(other)
    assert '"a // b"' in bench._code_only(src)  # text inside a string literal is code


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    h = bench.kernel_sources_hash()
    (tmp_path / "traffic.json").write_text(json.dumps({
        "label": {"source_hash": h, "bytes_per_launch": 123},
        "row": {"source_hash": "0" * 16, "bytes_per_launch": 456}}))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.traffic_from_profile("label", h) == 123
    assert bench.traffic_from_profile("row", h) is None  # taken on other sources
    assert bench.traffic_from_profile("finish", h) is None  # not measured


def test_algorithmic_bytes_of_the_large_sbm():
    # row pointers 4(n+1), index + value 8 per entry, one byte of labels per node, Q written 4nK
    n, nnz, K = 2_000_000, 48_002_260, 5
    assert bench.label_pass_bytes(n, nnz, K, 4) == 4 * (n + 1) + 8 * nnz + n + 4 * n * K == 434_018_084
    assert bench.iteration_bytes(n, nnz, K, 4, 4) == 4 * (n + 1) + 8 * nnz + 2 * n * K * 4 + 3 * n
