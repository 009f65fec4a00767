"""D3Q19 velocity set and weights (oracle copy; test infrastructure only).

Order: 0 rest; 1-6 = +x, -x, +y, -y, +z, -z; 7-18 = the 12 edge vectors in
opposite pairs (7, 8), (9, 10), ..., (17, 18).  Weights 1/3, 1/18, 1/36
(Sec. 3: the velocity set and its weights fix the moments of Eq. (8)).
"""
C19 = (
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
)
W19 = (1.0 / 3.0,) + (1.0 / 18.0,) * 6 + (1.0 / 36.0,) * 12
OPP = tuple(0 if i == 0 else (i + 1 if i % 2 == 1 else i - 1) for i in range(19))
