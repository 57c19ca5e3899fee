"""bench.py's command-line contract on the host (no GPU work is started)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_workload_configs():
    sys.path.insert(0, ROOT)
    import bench
    cfg = bench.configs()
    assert set(cfg) == {"c1", "c2", "c2x2", "c2x4", "c3", "c4", "c5", "control64", "slab2", "slab4", "slab8"}
    for g in (2, 4, 8):
        assert cfg["slab%d" % g]["dims"] == [(32, 32, 32, 32 // g)] and cfg["slab%d" % g]["betas"] == [2.6]
    for r in (2, 4):
        assert cfg["c2x%d" % r]["dims"] == [(32, 32, 32, 32)] * r and cfg["c2x%d" % r]["betas"] == [2.6] * r
    assert cfg["c2"]["dims"] == [(32, 32, 32, 32)] and cfg["c2"]["betas"] == [2.6]
    assert cfg["c1"]["dims"] == [(8, 8, 8, 8)] and cfg["c1"]["seed"] == 1
    assert len(cfg["c3"]["dims"]) == 16 and len(cfg["c5"]["dims"]) == 64
    for c in cfg.values():
        assert all(all(n % 2 == 0 for n in d) for d in c["dims"])


def test_every_global_name_is_defined():
    """Every name that a function of bench.py reads as a global exists at
    module level or among the builtins (a renamed or deleted helper fails
    here rather than on the GPU)."""
    import builtins
    import symtable
    src = open(os.path.join(ROOT, "bench.py")).read()
    top = symtable.symtable(src, "bench.py", "exec")
    defined = {s.get_name() for s in top.get_symbols() if s.is_assigned() or s.is_imported()}
    defined |= set(dir(builtins))
    missing = []

    def walk(t):
        for child in t.get_children():
            if child.get_type() == "function":
                for s in child.get_symbols():
                    if s.is_global() and s.is_referenced() and s.get_name() not in defined:
                        missing.append((child.get_name(), s.get_name()))
            walk(child)
    walk(top)
    assert not missing, missing


def test_traffic_lookup_grid():
    """The stored fabric traffic is keyed by the workgroups that take tiles:
    grid 0 and persistent grids at or beyond the (rounded) tile count hand
    out the same tiles to the same XCDs."""
    sys.path.insert(0, ROOT)
    import bench
    tiles = (32 ** 4 // 2) // 256                       # 32^4, block 256, one link per lane
    assert bench.effective_grid(0, tiles) == bench.effective_grid(4096, tiles) == 2048
    assert bench.effective_grid(1024, tiles) == 1024    # several tiles per workgroup: its own key
    assert bench.effective_grid(0, 5) == 8
    for key in bench.HB_TRAFFIC["by_launch"]:
        block, grid, _, nl = key
        assert bench.effective_grid(grid, (32 ** 4 // 2) // (block * nl)) == grid


def test_source_hash_ignores_comments_only():
    """The traffic table is keyed by the code of the kernel sources: comments
    and layout do not change the key, code (string literals included) does."""
    sys.path.insert(0, ROOT)
    import bench
    a = 'int a = 1; // one\n/* two\n lines */ const char *s = "x // y";\n'
    b = 'int   a = 1;\n\n const char *s = "x // y"; /* other */\n'
    c = 'int a = 2; const char *s = "x // y";\n'
    d = 'int a = 1; const char *s = "x /* y";\n'
    assert bench.code_only(a) == bench.code_only(b) == 'int a = 1; const char *s = "x // y";'
    assert bench.code_only(c) != bench.code_only(a)
    assert bench.code_only(d) != bench.code_only(a)
    assert bench.code_only("char q = '\"'; // \"\nint z;") == "char q = '\"'; int z;"
