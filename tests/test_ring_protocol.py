"""Model of the cross-workgroup boundary ring (engine.hpp, x_pull / x_room /
x_push): the producer publishes each 32-frame block's values into a ring of
512 slots as soon as the consumer's released count allows, the consumer pulls
a block's values plus the next block's first one.  Run with the producer as
far ahead as the protocol allows, no slot the consumer still needs may be
overwritten.  The release count the consumer stores must exclude the value
its next pull starts with (a release of i0 + cnt instead of i0 + cnt - 1 let
the producer overwrite it when the ring ran full)."""
RING = 512
BLK = 32


def run(T, release_last):
    ring = {}                       # slot -> value index held
    cons = 0                        # values below cons may be overwritten
    pushed = 0                      # values 0 .. pushed-1 are in the ring
    nsteps = T - 1
    nblk = (nsteps + BLK - 1) // BLK

    def push_until_blocked():
        # value 0 before the first block, then block k: values 32k+1 .. 32k+n
        nonlocal pushed
        if pushed == 0:
            ring[0] = 0
            pushed = 1
        while pushed < T:
            k = (pushed - 1) // BLK
            i_end = pushed + min(BLK, nsteps - BLK * k)
            if i_end - RING > cons:             # x_room: the slots are not released yet
                return
            for v in range(pushed, i_end):
                ring[v % RING] = v
            pushed = i_end

    for b in range(nblk):
        n = min(BLK, nsteps - BLK * b)
        push_until_blocked()
        need = range(BLK * b, BLK * b + n + 1)     # the block plus one value ahead
        assert pushed >= BLK * b + n + 1
        for v in need:
            if ring.get(v % RING) != v:
                return False
        cons = BLK * b + n + 1 - (1 if release_last else 0)
    return True


def test_ring_never_overwrites_a_needed_value():
    for T in (2, 33, 513, 545, 1000, 5000, 90000):
        assert run(T, release_last=True)


def test_releasing_the_next_first_value_breaks_the_ring():
    # the former release count: the producer runs 512 values ahead and
    # overwrites the value the next pull starts with
    assert not run(5000, release_last=False)
