"""The index arithmetic behind the class-major apply stream, checked on full
enumerations with the oracle's hash (Eq. TotalCost), independently of the
kernels:

* rows of one run (one particle moved between orbitals 0 and 1 per step)
  have consecutive indices and share g + n_0, and no two runs share it;
* a jump's target moves with the row along a run: if two jumps change the
  prefix sums S_1 .. S_{M-2} alike (one class) and their S_0 changes differ
  by s, the second's target at row g is the first's target at row g + s
  (same run) and the first's target at g plus s;
* slots reaching one configuration: the first in slot order (the row
  itself, the single jump, or the pair of a true double jump) removes a
  subset of what the others remove, so it is possible wherever they are.
"""

import pytest

from oracle import combinatorics as cb


def slots(M, form):
    """(removals, creations) of the row itself, the single jumps, then the
    double jumps of the form, in the order the apply streams them."""
    out = [((), ())]
    out += [((a,), (b,)) for a in range(M) for b in range(M) if a != b]
    for k in range(M):
        for s in range(k, M):
            for q in range(M):
                for l in range(M):
                    if form == "reduced" and (q > l or q in (k, s) or l in (k, s)):
                        continue
                    out.append(((k, s), (q, l)))
    return out


def prefix_change(M, rem, add):
    return tuple(sum(a <= m for a in add) - sum(r <= m for r in rem) for m in range(M - 1))


def move(n, rem, add):
    n = list(n)
    for r in rem:
        if n[r] == 0:
            return None
        n[r] -= 1
    for a in add:
        n[a] += 1
    return n


def space(N, M):
    D = cb.dim(N, M)
    return D, [cb.config_of(g, N, M) for g in range(D)]


@pytest.mark.parametrize("N,M", [(6, 3), (7, 4), (6, 5), (4, 6)])
def test_run_keys(N, M):
    D, occ = space(N, M)
    keys = [g + occ[g][0] for g in range(D)]
    for g in range(D):
        if occ[g][0] > 0:
            # the next index moves one particle from orbital 0 to 1
            nxt = list(occ[g])
            nxt[0] -= 1
            nxt[1] += 1
            assert occ[g + 1] == nxt
    for g in range(D):
        for h in range(D):
            assert (keys[g] == keys[h]) == (occ[g][2:] == occ[h][2:])


@pytest.mark.parametrize("form", ["reduced", "paper"])
@pytest.mark.parametrize("N,M", [(7, 3), (6, 4), (5, 5), (4, 6)])
def test_member_targets_follow_the_anchor(N, M, form):
    D, occ = space(N, M)
    keys = [g + occ[g][0] for g in range(D)]
    sl = slots(M, form)
    classes = {}
    for rem, add in sl:
        d = prefix_change(M, rem, add)
        classes.setdefault(d[1:], []).append((d[0], rem, add))
    checked = 0
    for members in classes.values():
        d0a, rema, adda = members[0]
        for d0, rem, add in members[1:]:
            s = d0a - d0
            for g in range(D):
                tm = move(occ[g], rem, add)
                if tm is None:
                    continue
                tm = cb.index_of(tm)
                ta = move(occ[g], rema, adda)
                if ta is not None:
                    assert tm == cb.index_of(ta) + s
                    checked += 1
                h = g + s
                if 0 <= h < D and keys[h] == keys[g]:
                    th = move(occ[h], rema, adda)
                    if th is not None:
                        assert tm == cb.index_of(th)
                        checked += 1
    assert checked > 0


@pytest.mark.parametrize("form", ["reduced", "paper"])
@pytest.mark.parametrize("M", [3, 4, 5, 6])
def test_group_leader_is_possible_wherever_its_slots_are(M, form):
    groups = {}
    for rem, add in slots(M, form):
        groups.setdefault(prefix_change(M, rem, add), []).append(rem)
    for rems in groups.values():
        lead = sorted(rems[0])
        for rem in rems[1:]:
            rest = list(rem)
            for r in lead:
                assert r in rest
                rest.remove(r)
    # the reduced form's slots all reach different configurations
    if form == "reduced":
        assert all(len(r) == 1 for r in groups.values())
