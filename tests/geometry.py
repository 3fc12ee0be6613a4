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


def stream_blocks_2d(I0, r, chunk, xcds=8):
    """Output-row ranges [a, b) of a 2D launch's stream blocks.  The rows form
    nb bands of ceil(I0 / nb) rows, nb = 8 or the largest of 4, 2, 1 whose
    bands still hold one block of h_SN rows.  A band holds blocks of
    h = min(chunk, band) rows; when it has room for more than two of them
    (and h >= 32), its last rows go in blocks of h // 2, so each XCD ends on
    short blocks."""
    h = max(1, chunk)
    nb = xcds
    while nb > 1 and -(-I0 // nb) < h:
        nb //= 2
    hb = -(-I0 // nb)
    h1 = max(1, min(h, hb))
    if hb // h1 > 2 and h1 >= 32:
        n1, h2 = hb // h1 - 2, h1 // 2
    else:
        n1, h2 = 0, h1
    out = []
    for x in range(nb):
        lo, hi = r + x * hb, min(r + (x + 1) * hb, I0 + r)
        a = lo
        for _ in range(n1):
            if a >= hi:
                break
            out.append((a, min(a + h1, hi)))
            a += h1
        while a < hi:
            out.append((a, min(a + h2, hi)))
            a += h2
    return out
