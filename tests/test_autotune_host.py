"""Host checks of the autotuner's candidate shapes."""
from paper_1907_06487_amd import autotune


def test_candidates_worker_counts_and_expanded_choice():
    c = autotune.candidates(400000, 1, 512)
    assert [d["n_workers"] for d in c] == [50, 100, 200]
    assert all(d["low_locality"] == "race" and d["window_max"] == autotune.max_window(1) for d in c)
    c = autotune.candidates(400000, 4, 512, window=3840, low_locality="auto")
    assert [d["low_locality"] for d in c] == ["auto", "auto", "auto", "expanded"]
    assert [d["low_locality"] for d in autotune.candidates(400000, 1, 512, low_locality="auto")] == ["auto"] * 3
    assert c[-1]["n_workers"] == 100 and all(d["window_max"] == 3840 for d in c)
    assert [d["n_workers"] for d in autotune.candidates(10, 1, 256)] == [4]


def test_max_window_fits_the_lds():
    for k in (1, 2, 4, 8, 16):
        w = autotune.max_window(k)
        assert w * (16 * k + 4) <= 159 * 1024
    assert autotune.max_window(1) == 3840
