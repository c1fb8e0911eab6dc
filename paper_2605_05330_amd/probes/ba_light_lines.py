"""Input of the gather-rate probe (gather_rate.hip): the light rows (degree <= 16)
of the Barabasi-Albert benchmark graph (n = 200,000, m = 5, seed 0) as sliced
lines, int32 [S][16][64], rows in degree-descending order, padding = n (a zero
slot).  Usage: python ba_light_lines.py OUTDIR  (writes OUTDIR/ba_lines.bin)."""
import os
import sys
import numpy as np
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from paper_2605_05330_amd import inputs as I
g = I.barabasi_albert(200_000, 5, 0)
deg = np.diff(g.row_ptr)
order = np.argsort(-deg, kind='stable')
inv = np.empty_like(order); inv[order] = np.arange(g.n)
light = [r for r in order if deg[r] <= 16]
S = (len(light) + 63) // 64
lines = np.full((S, 16, 64), g.n, dtype=np.int32)
for k, r in enumerate(light):
    s, l = divmod(k, 64)
    cols = inv[g.col_idx[g.row_ptr[r]:g.row_ptr[r + 1]]]
    lines[s, :len(cols), l] = cols
out = sys.argv[1]
lines.tofile(out + '/ba_lines.bin')
print('n', g.n, 'light rows', len(light), 'slices', S, 'gathers', int(deg[deg <= 16].sum()), 'all nnz', g.nnz)
