"""The profile tooling on the CPU: the code hash that stamps traffic records
ignores comments and whitespace but not code."""
from paper_1705_02257_amd import profiling


def test_code_only_drops_comments_keeps_code_and_strings():
    a = "int x = 1; // note\n/* block\n comment */ const char* s = \"a // b\";\n"
    b = "int x=1;\n\n   const char* s = \"a // b\"; // other note\n"
    assert profiling._code_only(a) == profiling._code_only(b)
    assert profiling._code_only(a) != profiling._code_only(a.replace("x = 1", "x = 2"))
    assert "a // b" in profiling._code_only(a)


def test_source_sha_is_stable_under_comment_edits(tmp_path):
    src = tmp_path / "k.hpp"
    src.write_text("__global__ void f(int* p) { p[0] = 1; }  // one\n")
    h1 = profiling.source_sha([str(src)])
    src.write_text("// header\n__global__ void f(int* p) {\n  p[0] = 1;  /* two */\n}\n")
    assert profiling.source_sha([str(src)]) == h1
    src.write_text("__global__ void f(int* p) { p[0] = 2; }\n")
    assert profiling.source_sha([str(src)]) != h1
