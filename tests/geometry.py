"""The library's tile geometry along the last axis, restated for the tests
(sizing grids to span several tiles plus a ragged tail; brute-force counts of
the performance model)."""


def overlap_left(bt, r, elem):
    """Overlap columns on a tile's left: >= bt*r, and (x - r) a multiple of
    16 bytes / elem, so every tile starts on the same 16-byte phase."""
    x = bt * r
    while (x - r) % (16 // elem):
        x += 1
    return x


def overlap_right(bt, r, elem):
    y = bt * r
    while (overlap_left(bt, r, elem) + y) % (16 // elem):
        y += 1
    return y


def compute_width(w, bt, r, elem):
    return w - overlap_left(bt, r, elem) - overlap_right(bt, r, elem)
