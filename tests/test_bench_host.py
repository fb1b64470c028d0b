"""Host-side helpers of bench.py (no GPU): the counter-summary lookup and the
tuning-cache bucket rule."""
import bench


def write_summary(path, workload, sha, tuned, nbytes):
    lines = ["# a counter summary", f"workload: {workload}", f"kernel_source_sha1: {sha}"]
    if tuned is not None:
        lines.append(f"tuned: {tuned}")
    lines.append(f"hbm_bytes_per_step: {nbytes}")
    path.write_text("\n".join(lines) + "\n")


def test_measured_traffic_needs_workload_sources_and_launch_choice(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    sha = bench.kernel_source_hash()
    write_summary(tmp_path / "xcorr_dish_counters.txt", "dish", sha, "N=32: 16-row ring split 1", 4369469629)
    assert bench.measured_traffic("dish", "N=32: 16-row ring split 1") == 4369469629.0
    # another launch choice, another workload's file, other kernel sources: no figure
    assert bench.measured_traffic("dish", "N=32: 32-row ring split 2") is None
    assert bench.measured_traffic("cylinder", "N=32: 16-row ring split 1") is None
    write_summary(tmp_path / "xcorr_dish_counters.txt", "dish", "0" * 16, "N=32: 16-row ring split 1", 1)
    assert bench.measured_traffic("dish", "N=32: 16-row ring split 1") is None
    # a summary keyed by another workload name inside the file
    write_summary(tmp_path / "xcorr_dish_counters.txt", "cylinder", sha, "N=32: 16-row ring split 1", 1)
    assert bench.measured_traffic("dish", "N=32: 16-row ring split 1") is None


def test_fstage_traffic_is_keyed_by_its_own_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    src = bench.FSTAGE_SOURCES["chan"]
    write_summary(tmp_path / "fstage_chan_counters.txt", "chan", bench.kernel_source_hash(src), None, 17817583740)
    assert bench.measured_traffic("chan", None, "fstage", src) == 17817583740.0
    # the X-engine's hash does not validate an F-stage summary
    write_summary(tmp_path / "fstage_chan_counters.txt", "chan", bench.kernel_source_hash(), None, 1)
    assert bench.measured_traffic("chan", None, "fstage", src) is None


def test_bucket_is_ceil_log2():
    assert [bench._bucket(v) for v in (1, 2, 3, 4, 5, 1024, 1025, 16384)] == [0, 1, 2, 2, 3, 10, 11, 14]
