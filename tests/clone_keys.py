"""Check of the crystal keys in a GPU track log against the oracle's key derivation."""
import numpy as np

import oracle


def check_clone_keys(lg, seed=0, n_clones=2):
    """Every finished track's crystal key is one of the keys its family can hold after the
    cloning depths it crossed (the oracle's primary-key and child-key derivation applied
    next_k times; Sec. 2: clones differ only in the material created after the cloning),
    its weight is n_clones^-next_k, and no two tracks of a family share a key."""
    levels = {}
    seen = set()
    for lin, nk, key, w in zip(lg["lineage"], lg["next_k"], lg["key"], lg["w"]):
        lin, nk, key = int(lin), int(nk), int(key)
        assert w == float(n_clones) ** -nk, (lin, nk, w)
        lv = levels.setdefault(lin, [np.array([oracle.primary_key(seed, lin)], np.uint64)])
        while len(lv) <= nk:
            lv.append(oracle.child_keys(lv[-1], seed, len(lv) - 1, n_clones))
        assert np.any(lv[nk] == np.uint64(key)), (lin, nk, hex(key))
        assert (lin, key) not in seen, (lin, hex(key))
        seen.add((lin, key))
    return len(levels)
