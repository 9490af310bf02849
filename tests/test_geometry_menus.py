"""Every trellis size the library accepts has a compiled layout: for the
batched kernel (S <= 4096, W in {1,2,4}) and for single launches
(S <= 32768), some (W, M) of the menus in tune.hpp covers S with the top
wave holding S-1 and S-2.  (A gap here once left utterances unprocessed.)"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_2310_17864_amd", "csrc", "tune.hpp")


def menu(name):
    txt = open(TUNE).read()
    m = re.search(name + r"\[\]\s*=\s*\{([^}]*)\}", txt)
    return [int(x) for x in m.group(1).split(",")]


def geo_ok(S, W, M):
    seg = 64 * M
    return W * seg >= S and (W == 1 or (W - 1) * seg + 2 <= S)


def test_pack_menu_covers_all_sizes():
    pack = menu("kMenuPack")
    gaps = [S for S in range(1, 4097) if not any(geo_ok(S, W, M) for W in (1, 2, 4) for M in pack)]
    assert gaps == []


def test_single_menus_cover_all_sizes():
    one, long_ = menu("kMenuOne"), menu("kMenuLong")
    gaps = [S for S in range(1, 32769)
            if not (any(geo_ok(S, W, M) for W in range(1, 5) for M in one)
                    or any(geo_ok(S, W, M) for W in range(1, 9) for M in long_))]
    assert gaps == []


def test_multi_menu_covers_long_single_launches():
    # single launches above 4096 states use the multi-workgroup layout: the
    # chooser takes W = ceil(S / (64 M)) for the first M of the menu that
    # holds S; every odd S (S = 2L + 1) up to 32768 must find one with W <= 256
    # (32 workgroups of 8 waves)
    multi = menu("kMenuMulti")
    gaps = [S for S in range(4097, 32769, 2)
            if not any(geo_ok(S, -(-S // (64 * M)), M) and -(-S // (64 * M)) <= 256 for M in multi)]
    assert gaps == []


def test_serve_menu_covers_large_requests():
    # the resident serving kernel runs trellises above the pack limit on one
    # 16-wave workgroup: the chooser takes the first M >= 8 of the pack menu
    # with W = ceil(S / (64 M)) <= 16 whose top wave holds S-1 (and S-2, or
    # else takes a(S-2) from the boundary ring); every odd S up to
    # 16 * 64 * 16 must find one
    pack = [m for m in menu("kMenuPack") if m >= 8]

    def top1_ok(S, W, M):
        seg = 64 * M
        return W * seg >= S and (W == 1 or (W - 1) * seg + 1 <= S)

    gaps = [S for S in range(4097, 16385, 2)
            if not any(top1_ok(S, -(-S // (64 * M)), M) and -(-S // (64 * M)) <= 16 for M in pack)]
    assert gaps == []
    # without the one-state top segment two sizes would have no layout
    strict = [S for S in range(4097, 16385, 2)
              if not any(geo_ok(S, -(-S // (64 * M)), M) and -(-S // (64 * M)) <= 16 for M in pack)]
    assert strict == [14337, 15361]


def test_serve_parts_menu():
    # large served requests may run over up to 4 resident workgroups of 16
    # waves with 4, 6 or 8 states per lane (the first M whose top segment
    # holds S-1 and S-2); sizes none of them fits keep the one-workgroup
    # layout, which covers every size (test above)
    parts = [4, 6, 8]
    none = [S for S in range(4097, 16385, 2)
            if not any(geo_ok(S, -(-S // (64 * M)), M) and -(-S // (64 * M)) <= 64 for M in parts)]
    assert all((S - 1) % 1536 == 0 for S in none)
    assert len(none) <= 8
