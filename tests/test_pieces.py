"""The row-piece cut of the fused launches (paper_2405_12631_amd/csrc/wv_pieces.h): the cap it
chooses against a plain simulation of the round-robin item deal, and the cut itself."""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CAPS = (16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 1024)


def seg_rows(h, cap):
    pieces = (h + cap - 1) // cap
    return (h + pieces - 1) // pieces


def simulated_cap(shapes, strip, fill, resident):
    """Deal every item (strip fastest, then piece, then plane, group after group) to
    workgroup k mod g one by one; the cap with the smallest busiest workgroup wins (first on
    ties)."""
    best, best_cap = None, 128
    for cap in CAPS:
        costs = []
        for h, w, n in shapes:
            sr = seg_rows(h, cap)
            sy = (h + sr - 1) // sr
            sx = (w + strip - 1) // strip
            for _ in range(n):
                for y in range(sy):
                    costs += [min(sr, h - y * sr) + fill] * sx
        if not costs:
            return 128
        g = min(len(costs), max(resident, 1))
        load = [0] * g
        for k, c in enumerate(costs):
            load[k % g] += c
        worst = max(load)
        if best is None or worst < best:
            best, best_cap = worst, cap
    return best_cap


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("pieces") / "pieces_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "pieces_driver.cpp")], check=True)
    return exe


def test_cut_is_even_and_bounded():
    for h in range(1, 1200):
        for cap in CAPS:
            r = seg_rows(h, cap)
            pieces = (h + r - 1) // r
            assert 1 <= r <= cap and pieces == (h + cap - 1) // cap
            assert h - (pieces - 1) * r >= 1   # the last piece is not empty


def test_chosen_cap_matches_item_deal_simulation(driver):
    rng = random.Random(7)
    dims = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 136, 192, 256, 272, 384, 480, 544, 960]
    launches = []
    for _ in range(400):
        shapes = [(rng.choice(dims), rng.choice(dims), rng.randrange(0, 40)) for _ in range(rng.randint(1, 4))]
        launches.append((rng.choice((58, 64)), rng.choice((3, 10)), rng.choice((80, 256, 304)), shapes))
    # the 64-image batch's level-1 subbands (step stack and ConvLSTM launches)
    batch = [(128, 128, 54), (256, 384, 54), (512, 512, 45), (544, 960, 39)]
    launches += [(58, 10, 256, batch), (64, 3, 256, batch)]
    text = "".join(f"{s} {f} {r} {len(sh)} " + " ".join(f"{h} {w} {n}" for h, w, n in sh) + "\n"
                   for s, f, r, sh in launches)
    out = subprocess.run([driver], input=text, capture_output=True, text=True, check=True).stdout.split()
    assert len(out) == len(launches)
    for (s, f, r, sh), got in zip(launches, out):
        assert int(got) == simulated_cap(sh, s, f, r), (s, f, r, sh)
