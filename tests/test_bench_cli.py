"""bench.py's command line on the CPU: it measures one GPU and says so for
any other count, before touching a device; its host-only subcommands turn
counter folders into the traffic record's numbers."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 4" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_csv_reader_orders_dispatches(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    d = tmp_path / "pmc"
    d.mkdir()
    (d / "pmc_counter_collection.csv").write_text(
        '"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n'
        '3,"k3","FETCH_SIZE",30\n1,"k1","FETCH_SIZE",10\n2,"k2","WRITE_SIZE",5\n2,"k2","FETCH_SIZE",20\n')
    assert bench._read_counter_csv(str(tmp_path), "FETCH_SIZE") == [("k1", 10.0), ("k2", 20.0), ("k3", 30.0)]
    assert bench._read_counter_csv(str(tmp_path), "WRITE_SIZE") == [("k2", 5.0)]
