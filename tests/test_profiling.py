"""The profile tooling on the CPU: the code hash that stamps traffic records
ignores comments and whitespace but not code, and the SQ-counter shares
follow from the counter sums and dispatch durations."""
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


def test_sq_shares_from_a_synthetic_run(tmp_path):
    """Two dispatches of one kernel, 1 ms each (4.8e6 cycles at 2.4 GHz):
    the shares follow from the counter sums and the durations alone."""
    import csv
    from paper_1705_02257_amd.profiling import sq_table
    cyc = 2.4e6                              # one dispatch of 1 ms
    rows = []
    for disp in ("1", "2"):
        for name, per_cu_cycle in (("SQ_INSTS_VALU", 0.25), ("SQ_LDS_BANK_CONFLICT", 0.1),
                                   ("SQ_INSTS_LDS", 0.05), ("SQ_WAIT_INST_LDS", 0.32)):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": "void ips4o::k_classify<0, 1024, 8>(ips4o::Ctx<0>)",
                         "Counter_Name": name, "Counter_Value": str(per_cu_cycle * 256 * cyc),
                         "Start_Timestamp": "1000000", "End_Timestamp": "2000000"})
    rows.append({"Dispatch_Id": "3", "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "SQ_INSTS_VALU",
                 "Counter_Value": "5", "Start_Timestamp": "0", "End_Timestamp": "10"})
    with open(tmp_path / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)
    t = sq_table(str(tmp_path))
    assert list(t) == ["k_classify<0, 1024, 8>"]
    v = t["k_classify<0, 1024, 8>"]
    assert v["dispatches"] == 2 and abs(v["ms"] - 2.0) < 1e-12
    assert abs(v["conflict"] - 0.1) < 1e-12          # per CU-cycle
    assert abs(v["valu"] - 0.25) < 1e-12             # 4 cycles per instruction over 4 SIMDs
    assert abs(v["ldswait"] - 0.32 / 16) < 1e-12     # 16 resident waves per CU
