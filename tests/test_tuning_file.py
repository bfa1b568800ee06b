"""The autotuner's cache file (host only, no GPU needed): entries loaded from a file come back
unchanged from a save, and malformed or out-of-range files are rejected before anything is
loaded."""
import json

import pytest

from paper_2306_17537_amd import ie

ARCH = "gfx950:test-only"


def _entry(grid=(33, 20, 17), fft=(96, 48, 48), prec="c128", var=(1, 2, 5, 3, 0)):
    return {"arch": ARCH, "precision": prec, "grid": list(grid), "fft": list(fft),
            "variant": list(var),
            "us": [[round(10.0 + q + 0.25 * v, 2) for v in range(8)] for q in range(5)]}


def _ours(entries):
    return sorted((e for e in entries if e["arch"] == ARCH),
                  key=lambda e: (e["precision"], e["grid"], e["fft"]))


def test_load_then_save_round_trip(tmp_path):
    want = [_entry(), _entry(prec="c64", var=(0, 3, 7, 1, 1)),
            _entry(grid=(48, 48, 64), fft=(128, 128, 128), var=(1, 3, 4, 0, 1))]
    src = tmp_path / "in.json"
    src.write_text(json.dumps(want, indent=2))
    ie.ie_tuning_load(str(src))
    out = tmp_path / "out.json"
    ie.ie_tuning_save(str(out))
    got = json.loads(out.read_text())
    assert _ours(got) == _ours(want)


@pytest.mark.parametrize("bad", [
    lambda e: e.pop("variant"),
    lambda e: e.__setitem__("variant", [0, 0, 8, 0, 0]),     # x pass has variants 0..7
    lambda e: e.__setitem__("variant", [0, 4, 0, 0, 0]),     # y passes 0..3
    lambda e: e.__setitem__("variant", [2, 0, 0, 0, 0]),     # z passes 0..1
    lambda e: e.__setitem__("fft", [64, 48, 48]),            # 64 < 2 * 33 - 1
    lambda e: e.__setitem__("fft", [192, 48, 48]),           # not a length the library picks
    lambda e: e.__setitem__("precision", "bf16"),
    lambda e: e.__setitem__("grid", [0, 20, 17]),
    lambda e: e.__setitem__("us", [[1.0] * 8] * 4),
])
def test_malformed_files_are_rejected_whole(tmp_path, bad):
    good = _entry(grid=(5, 7, 3), fft=(16, 16, 8))
    e = _entry(grid=(9, 9, 9), fft=(24, 24, 24))
    bad(e)
    src = tmp_path / "bad.json"
    src.write_text(json.dumps([good, e]))
    with pytest.raises(ie.IEError) as err:
        ie.ie_tuning_load(str(src))
    assert err.value.code == ie.IE_EINVAL
    out = tmp_path / "out.json"
    ie.ie_tuning_save(str(out))
    assert not any(x["grid"] == [5, 7, 3] for x in _ours(json.loads(out.read_text())))


def test_unreadable_paths_are_rejected(tmp_path):
    with pytest.raises(ie.IEError):
        ie.ie_tuning_load(str(tmp_path / "missing.json"))
    with pytest.raises(ie.IEError):
        ie.ie_tuning_save(str(tmp_path / "no-such-dir" / "x.json"))
    src = tmp_path / "text.json"
    src.write_text("not json")
    with pytest.raises(ie.IEError):
        ie.ie_tuning_load(str(src))
