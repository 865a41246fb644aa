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
