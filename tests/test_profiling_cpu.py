"""Host-side checks of the profiling helpers that stamp and read the committed
rocprofv3 summaries: the code hash ignores comments and blank lines but not
code, and the HBM-traffic scaling divides by what the counters read for a
copy of known size."""
import csv

from paper_2511_21660_amd import profiling as P


def test_code_hash_ignores_comments_not_code():
    src = "int a = 1;  // one\n/* block\n comment */\n\nint b = a + 2;\n"
    assert P._code_only(src) == P._code_only("int a = 1;\nint b = a + 2;  // two\n")
    assert P._code_only(src) != P._code_only("int a = 1;\nint b = a + 3;\n")
    assert P._code_only("x = 1; /* a */ y = 2; /* b\n c */ z = 3;") == "x = 1;  y = 2;  z = 3;"
    h = P.source_hash()
    assert len(h) == 16 and int(h, 16) >= 0 and h == P.source_hash()


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_scaled_by_the_copy_kernel(tmp_path):
    """A copy kernel moving 1000 B each way reads FETCH 500 and WRITE 1000: the
    decode kernel's readings are scaled by 2 and 1."""
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(fetch, [{"Kernel_Name": "void at::bitwise_not_kernel", "Counter_Name": "FETCH_SIZE",
                          "Counter_Value": 1000 / 2 / 1024},
                         {"Kernel_Name": "rb::relay_block_kernel<1>", "Counter_Name": "FETCH_SIZE",
                          "Counter_Value": 300 / 1024}])
    _counter_csv(write, [{"Kernel_Name": "void at::bitwise_not_kernel", "Counter_Name": "WRITE_SIZE",
                          "Counter_Value": 1000 / 1024},
                         {"Kernel_Name": "rb::relay_block_kernel<1>", "Counter_Name": "WRITE_SIZE",
                          "Counter_Value": 50 / 1024}])
    t = P.traffic(str(fetch), str(write), "relay_block_kernel", "bitwise_not", 1000)
    assert abs(t["fetch_scale"] - 2.0) < 1e-9 and abs(t["write_scale"] - 1.0) < 1e-9
    assert abs(t["fetch_bytes_per_launch"] - 600.0) < 1e-6
    assert abs(t["write_bytes_per_launch"] - 50.0) < 1e-6
    assert abs(t["traffic_bytes_per_launch"] - 650.0) < 1e-6
    assert t["source_hash"] == P.source_hash()
