"""The batch journal's host side, through the C ABI (no GPU call).

The journal holds one record per finished mock of a covariance batch (the
many realisations whose modal coefficients give the estimator's covariance,
Sec. 3.5 closing remark) so that a stopped batch resumes without redoing
them. These tests pin the on-disk format (a record written here byte by byte,
with its FNV-1a 64 checksum computed here, is read back by the library), the
matching rules, the repair of a torn tail, the detection of corruption, the
file lock, and that a writer killed with SIGKILL at random moments never
leaves anything but whole records in the valid prefix.
"""
import fcntl
import os
import signal
import struct
import subprocess
import sys
import time

import numpy as np
import pytest

import paper_1708_05303_amd as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fnv1a64(data: bytes) -> int:
    h = 0xcbf29ce484222325
    for c in data:
        h ^= c
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def record_bytes(key, chash, np_, Bm, alpha, beta):
    nl, ntri = Bm.shape
    head = struct.pack("<IIQQqiiii", 0x43455242, 0 if beta is None else 1, key, chash, np_, nl, ntri, alpha.size, 0)
    body = head + Bm.astype("<f8").tobytes() + alpha.astype("<f8").tobytes()
    if beta is not None:
        body += beta.astype("<f8").tobytes()
    return body + struct.pack("<Q", fnv1a64(body))


FILE_HEAD = b"BSPJRNL\x00" + struct.pack("<II", 1, 0)


def sample(seed, nl=3, ntri=7, d=12):
    r = np.random.default_rng(seed)
    return r.standard_normal((nl, ntri)), r.standard_normal(d), r.standard_normal(d)


def err_status(excinfo):
    return excinfo.value.status


def test_library_reads_a_record_written_by_hand(tmp_path):
    """The documented layout and checksum: a file assembled here is read back."""
    path = tmp_path / "hand.bspj"
    recs = [(11, 0xABCDEF0123456789, 5000, *sample(1)), (12, 0xABCDEF0123456789, 5100, *sample(2)[:2], None)]
    path.write_bytes(FILE_HEAD + b"".join(record_bytes(*r) for r in recs))
    assert B.bsp_journal_scan(str(path)) == (2, path.stat().st_size, path.stat().st_size)
    got = B.bsp_journal_lookup(str(path), 11, 0xABCDEF0123456789, 5000, 3, 7, 12)
    assert got is not None
    for a, b in zip(got, recs[0][3:]):
        assert np.array_equal(a, b)
    # a record without beta serves only callers that do not ask for beta
    assert B.bsp_journal_lookup(str(path), 12, 0xABCDEF0123456789, 5100, 3, 7, 12) is None
    got = B.bsp_journal_lookup(str(path), 12, 0xABCDEF0123456789, 5100, 3, 7, 12, with_beta=False)
    assert got is not None and np.array_equal(got[0], recs[1][3]) and np.array_equal(got[1], recs[1][4])


def test_library_writes_the_documented_layout(tmp_path):
    path = tmp_path / "lib.bspj"
    Bm, al, be = sample(3)
    B.bsp_journal_append(str(path), 77, 0x1234, 4242, Bm, al, be)
    assert path.read_bytes() == FILE_HEAD + record_bytes(77, 0x1234, 4242, Bm, al, be)


def test_matching_rules(tmp_path):
    path = str(tmp_path / "m.bspj")
    Bm, al, be = sample(4)
    B.bsp_journal_append(path, 5, 100, 900, Bm, al, be)
    assert B.bsp_journal_lookup(path, 5, 101, 900, 3, 7, 12) is None  # another configuration
    assert B.bsp_journal_lookup(path, 6, 100, 900, 3, 7, 12) is None  # another mock
    with pytest.raises(B.BspError) as e:  # same mock and configuration, another catalogue size
        B.bsp_journal_lookup(path, 5, 100, 901, 3, 7, 12)
    assert err_status(e) == 1
    with pytest.raises(B.BspError) as e:  # recorded twice
        B.bsp_journal_append(path, 5, 100, 900, Bm, al, be)
    assert err_status(e) == 1
    B.bsp_journal_append(path, 5, 101, 900, Bm, al, be)  # same key, another configuration
    assert B.bsp_journal_scan(path)[0] == 2


def test_last_record_of_a_key_wins(tmp_path):
    """A record written without beta, then the same mock recorded again with
    beta (what a batch that needs beta appends): lookups see the later one."""
    path = tmp_path / "w.bspj"
    Bm, al, be = sample(8)
    B.bsp_journal_append(str(path), 3, 50, 700, Bm, al, None)
    with open(path, "ab") as fh:
        fh.write(record_bytes(3, 50, 700, Bm + 1, al + 1, be))
    got = B.bsp_journal_lookup(str(path), 3, 50, 700, 3, 7, 12)
    assert got is not None
    assert np.array_equal(got[0], Bm + 1) and np.array_equal(got[1], al + 1) and np.array_equal(got[2], be)
    assert B.bsp_journal_scan(str(path))[0] == 2


def test_torn_tail_is_ignored_then_cut(tmp_path):
    path = tmp_path / "t.bspj"
    for k in range(4):
        B.bsp_journal_append(str(path), k, 9, 10 + k, *sample(k))
    full = path.read_bytes()
    rec = (len(full) - 16) // 4
    for cut in (1, 8, 47, 48, 49, rec // 2, rec - 8, rec - 1):
        path.write_bytes(full[:len(full) - cut])
        n, valid, size = B.bsp_journal_scan(str(path))
        assert (n, valid, size) == (3, 16 + 3 * rec, len(full) - cut), cut
        assert B.bsp_journal_lookup(str(path), 3, 9, 13, 3, 7, 12) is None
    # the next append cuts the torn record off and writes a whole one
    B.bsp_journal_append(str(path), 3, 9, 13, *sample(3))
    assert path.read_bytes() == full


def test_corruption_stops_the_valid_prefix(tmp_path):
    path = tmp_path / "c.bspj"
    for k in range(3):
        B.bsp_journal_append(str(path), k, 9, 10 + k, *sample(k))
    full = bytearray(path.read_bytes())
    rec = (len(full) - 16) // 3
    for off in (16 + rec + 20, 16 + rec + 100, 16 + 2 * rec - 3):  # key, payload, checksum of record 1
        bad = bytearray(full)
        bad[off] ^= 0x40
        path.write_bytes(bytes(bad))
        assert B.bsp_journal_scan(str(path))[:2] == (1, 16 + rec), off
    path.write_bytes(b"not a journal at all")
    with pytest.raises(B.BspError) as e:
        B.bsp_journal_scan(str(path))
    assert err_status(e) == 9
    with pytest.raises(B.BspError) as e:
        B.bsp_journal_scan(str(tmp_path / "absent.bspj"))
    assert err_status(e) == 9


def test_lock_refuses_a_second_writer(tmp_path):
    path = tmp_path / "l.bspj"
    B.bsp_journal_append(str(path), 1, 2, 3, *sample(0))
    with open(path, "rb") as fh:
        fcntl.flock(fh, fcntl.LOCK_EX)
        with pytest.raises(B.BspError) as e:
            B.bsp_journal_append(str(path), 2, 2, 3, *sample(1))
        assert err_status(e) == 9
        assert "locked" in str(e.value)
    B.bsp_journal_append(str(path), 2, 2, 3, *sample(1))
    assert B.bsp_journal_scan(str(path))[0] == 2


WRITER = r"""
import os
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import paper_1708_05303_amd as B
path = sys.argv[1]
k = B.bsp_journal_scan(path)[0] if os.path.exists(path) else 0
while True:
    Bm = np.full((3, 4000), float(k))
    B.bsp_journal_append(path, k, 7, 100 + k, Bm, np.full(150, float(k)), np.full(150, -float(k)))
    k += 1
"""


def test_writer_killed_at_random_moments_leaves_whole_records(tmp_path):
    """SIGKILL of a process that appends records as fast as it can, at random
    moments: every record in the valid prefix is whole and holds the values
    written for its key, and the next writer continues from there."""
    path = tmp_path / "k.bspj"
    script = tmp_path / "writer.py"
    script.write_text(WRITER)
    rng = np.random.default_rng(12)
    last = 0
    for trial in range(4):
        p = subprocess.Popen([sys.executable, str(script), str(path), ROOT], stdout=subprocess.DEVNULL,
                             stderr=subprocess.PIPE)
        time.sleep(1.0 + rng.uniform(0.0, 0.6))
        os.kill(p.pid, signal.SIGKILL)
        p.wait()
        # each writer resumed after the last whole record of the one before
        n, valid, size = B.bsp_journal_scan(str(path))
        assert n > last and valid <= size, (trial, n, last)
        last = n
        for k in sorted(set(rng.choice(n, size=min(n, 6), replace=False)) | {n - 1}):
            got = B.bsp_journal_lookup(str(path), int(k), 7, 100 + int(k), 3, 4000, 150)
            assert got is not None, (trial, k)
            assert np.all(got[0] == k) and np.all(got[1] == k) and np.all(got[2] == -k)
