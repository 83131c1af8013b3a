"""Word-size-generic Philox (Salmon et al., SC'11) in Python big-integer
arithmetic, written from the published description.  Its 4x64 instance is
checked against numpy's independent Philox4x64-10; its 4x32 instance is then
the reference for the oracle's (and the GPU's) Philox4x32-10."""

CONST = {
    32: dict(M=(0xD2511F53, 0xCD9E8D57), W=(0x9E3779B9, 0xBB67AE85)),
    64: dict(M=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
             W=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}


def philox4(ctr, key, bits=32, rounds=10):
    mask = (1 << bits) - 1
    M, W = CONST[bits]["M"], CONST[bits]["W"]
    c = [x & mask for x in ctr]
    k = [x & mask for x in key]
    for r in range(rounds):
        if r:
            k = [(k[0] + W[0]) & mask, (k[1] + W[1]) & mask]
        p0 = M[0] * c[0]
        p1 = M[1] * c[2]
        c = [(p1 >> bits) ^ c[1] ^ k[0], p1 & mask, (p0 >> bits) ^ c[3] ^ k[1], p0 & mask]
    return c
