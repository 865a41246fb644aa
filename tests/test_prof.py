"""CPU checks of the profile-record helpers: the source digest that ties a
measured-traffic record to the kernel code it was taken on."""
import json

from paper_2609_07387_amd import prof


def test_code_only_drops_comments_and_spacing_keeps_literals():
    a = 'int a = 1; // note\n/* block\n comment */ const char* s = "x // y /* z */"; char q = \'"\';'
    b = 'int  a = 1;\n\n const char* s = "x // y /* z */";   char q = \'"\';  // other note'
    assert prof._code_only(a) == prof._code_only(b)
    assert '"x // y /* z */"' in prof._code_only(a)
    assert prof._code_only("int a = 1;") != prof._code_only("int a = 2;")


def test_digest_follows_code_not_comments(tmp_path, monkeypatch):
    src = tmp_path / "csrc"
    src.mkdir()
    (src / "k.hip").write_text("__global__ void k(float* x) { x[0] = 1.f; }  // v1\n")
    monkeypatch.setattr(prof, "HERE", str(tmp_path))
    d1 = prof.source_digest()
    (src / "k.hip").write_text("// header comment\n__global__ void k(float* x) {\n    x[0] = 1.f;\n}\n")
    assert prof.source_digest() == d1
    (src / "k.hip").write_text("__global__ void k(float* x) { x[0] = 2.f; }\n")
    assert prof.source_digest() != d1


def test_stale_record_is_ignored(tmp_path, monkeypatch):
    src = tmp_path / "csrc"
    src.mkdir()
    (src / "k.hip").write_text("int k;\n")
    monkeypatch.setattr(prof, "HERE", str(tmp_path))
    rec = {"kernel": "k", "bytes_per_launch": 1.0, "source_digest": prof.source_digest()}
    md = tmp_path / "r.md"
    md.write_text("# r\n\n```json\n" + json.dumps(rec) + "\n```\n")
    assert prof.load_traffic(str(md))["bytes_per_launch"] == 1.0
    (src / "k.hip").write_text("int k2;\n")
    assert prof.load_traffic(str(md)) is None


def test_excluded_file_does_not_stale_a_record(tmp_path, monkeypatch):
    src = tmp_path / "csrc"
    src.mkdir()
    (src / "k.hip").write_text("int k;\n")
    (src / "other.hpp").write_text("int o;\n")
    monkeypatch.setattr(prof, "HERE", str(tmp_path))
    rec = {"kernel": "k", "bytes_per_launch": 1.0, "digest_exclude": ["other.hpp"],
           "source_digest": prof.source_digest(("other.hpp",))}
    md = tmp_path / "r.md"
    md.write_text("# r\n\n```json\n" + json.dumps(rec) + "\n```\n")
    (src / "other.hpp").write_text("int o2;\n")
    assert prof.load_traffic(str(md)) is not None
    (src / "k.hip").write_text("int k2;\n")
    assert prof.load_traffic(str(md)) is None


def _counter_csv(path, rows):
    """rows: (dispatch id, kernel name, counter, value)"""
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, k, c, v in rows:
            f.write(f"{d},{k},{c},{v}\n")


def test_request_size_estimate(tmp_path):
    """A copy of 1 MiB in 8192 requests (128 B each) and a kernel with 1000
    32-byte and 3000 other read requests: 32 000 + 3000 x 128 read bytes;
    writes: 100 of 64 B and 50 of 32 B."""
    mib = float(2 ** 20)
    rd = [(1, "copyBuffer", "TCC_EA0_RDREQ_sum", 8192), (1, "copyBuffer", "TCC_EA0_RDREQ_32B_sum", 0),
          (1, "copyBuffer", "TCC_BUBBLE_sum", 0), (1, "copyBuffer", "TCC_EA0_RDREQ_DRAM_sum", 8192)]
    wr = [(1, "copyBuffer", "TCC_EA0_WRREQ_sum", 16384), (1, "copyBuffer", "TCC_EA0_WRREQ_64B_sum", 16384),
          (1, "copyBuffer", "TCC_EA0_WRREQ_DRAM_sum", 16384)]
    for d in (2, 3):  # two dispatches of the kernel; the window takes the last
        f = 1 if d == 3 else 2
        rd += [(d, "kern", "TCC_EA0_RDREQ_sum", 4000 * f), (d, "kern", "TCC_EA0_RDREQ_32B_sum", 1000 * f),
               (d, "kern", "TCC_BUBBLE_sum", 0), (d, "kern", "TCC_EA0_RDREQ_DRAM_sum", 2000 * f)]
        wr += [(d, "kern", "TCC_EA0_WRREQ_sum", 150 * f), (d, "kern", "TCC_EA0_WRREQ_64B_sum", 100 * f),
               (d, "kern", "TCC_EA0_WRREQ_DRAM_sum", 150 * f)]
    _counter_csv(tmp_path / "r.csv", rd)
    _counter_csv(tmp_path / "w.csv", wr)
    z = prof.request_sizes(str(tmp_path / "r.csv"), str(tmp_path / "w.csv"), "kern", mib, n_last=1)
    assert z["copy_bytes_per_read_request"] == 128.0
    assert z["copy_write_bytes_from_sizes"] == mib
    assert z["read_bytes"] == 32_000 + 3000 * 128
    assert z["write_bytes"] == 100 * 64 + 50 * 32
    assert z["dram_read_share"] == 0.5
