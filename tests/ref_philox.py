"""Independent pure-Python Philox4x32-10 (Salmon et al., SC'11), big-integer arithmetic.

Used only to pin the oracle's C implementation and the GPU kernels' generator."""
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    x = [int(c) & MASK for c in ctr]
    k = [int(key[0]) & MASK, int(key[1]) & MASK]
    for r in range(10):
        if r:
            k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
        prod0 = M0 * x[0]
        prod1 = M1 * x[2]
        x = [(prod1 >> 32) ^ x[1] ^ k[0], prod1 & MASK, (prod0 >> 32) ^ x[3] ^ k[1], prod0 & MASK]
    return x
