"""The decoder's strides 4 and 2 run the stride-1 passes on the lattice of
that stride (coordinates s X, extent ceil(n / s)).  That rests on the edge
rules of the interpolation (Sec. 3.2, G-Interp: cubic where the neighbours
at -3s and +3s exist, linear where +s exists, else the copy of -s) being the
same at c = s X with extent n as at X with extent ceil(n / s) and stride 1.
Checked here exhaustively on small extents (host arithmetic only)."""


def _rule(c, n, s):
    if c >= 3 * s and c + 3 * s < n:
        return "cubic"
    if c + s < n:
        return "linear"
    return "copy"


def test_lattice_edge_rules_match_stride_one():
    for s in (1, 2, 4):
        for n in range(1, 300):
            big_n = (n + s - 1) // s
            for x in range(big_n):
                assert _rule(s * x, n, s) == _rule(x, big_n, 1), (s, n, x)


def test_lattice_extent_counts_the_points_below_n():
    for s in (1, 2, 4):
        for n in range(1, 300):
            assert (n + s - 1) // s == len(range(0, n, s))
