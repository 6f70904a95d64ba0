"""bench.py host-side behaviour (no GPU): the one-GPU guard and the counter
summary reader."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_summary_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "paper_2111_06868_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "mfma.hip").write_text("// kernel v1\n")
    sha = bench.source_hash(3)
    (prof / "traffic_mfma_f32_k5_30q.md").write_text(
        "- kernel_source_sha256_16: `%s`\n- hbm_bytes_per_launch: 17180946890\n" % sha)
    assert bench.read_traffic(3, 5, 30) == 17180946890.0
    (src / "mfma.hip").write_text("// kernel v2\n")
    assert bench.read_traffic(3, 5, 30) is None
    assert bench.read_traffic(3, 4, 30) is None


def test_plan_listing_covers_every_pass():
    """--plan lists the tiled plan of the 30-qubit grid circuit without a GPU:
    every pass's blocks lie inside its union, unions stay within the tile, and
    the blocks add up to the plan's block count."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--plan"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().splitlines()
    head = dict(kv.split("=") for kv in lines[0].split() if "=" in kv)
    assert head["n"] == "30" and head["gates"] == "845"
    rows = lines[1:]
    assert len(rows) == int(head["passes"])
    total = 0
    for row in rows:
        kind = row.split()[1]
        assert kind in ("tile", "single"), row
        fields = dict(kv.split("=", 1) for kv in row.split(None, 2)[2].replace(", ", ",").split() if "=" in kv)
        union = set(int(q) for q in fields["union"].strip("[]").split(","))
        blocks = [set(int(q) for q in b.split(",")) for b in row.split("blocks=")[1].split()]
        assert int(fields["s"]) == len(blocks)
        assert set().union(*blocks) == union
        assert all(1 <= len(b) <= 4 for b in blocks)
        # the tile (the union plus its lowest missing positions, 14 in all)
        # is made of runs of at least 2^4 amplitudes
        tile, p = set(union), 0
        while len(tile) < 14:
            tile.add(p)
            p += 1
        run = 0
        while run in tile:
            run += 1
        assert len(union) <= 14 and (len(union) <= 10 or run >= 4), row
        total += len(blocks)
    assert total == int(head["blocks"])
