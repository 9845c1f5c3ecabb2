"""The C ABI: every symbol declared in include/pic.h is exported by the built library, and
host-side validation (no device memory) rejects bad descriptors with the documented codes."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2501_07465_amd import pic
    L = pic.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(pic.EXPORTED) == set(names)


def test_create_validation_codes():
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    g = pic.grid_desc(w)
    g.tile[0] = 6  # not a power of two
    with pytest.raises(pic.PicError) as e:
        pic.pic_create(g)
    assert e.value.code == pic.PIC_EINVAL
    g = pic.grid_desc(w)
    g.dims = 4
    with pytest.raises(pic.PicError):
        pic.pic_create(g)


def test_cfl_rejected():
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    w["dt"] *= 1.1  # above the vacuum Courant limit
    h = pic.pic_create(pic.grid_desc(w))
    with pytest.raises(pic.PicError) as e:
        pic.pic_init_species(h, pic.species_desc(w["species"][0]), 1)
    assert e.value.code == pic.PIC_ECFL
    pic.pic_destroy(h)


def test_species_escaping_open_faces_rejected():
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    sp = dict(w["species"][0])
    sp["reflect"] = False
    h = pic.pic_create(pic.grid_desc(w))
    with pytest.raises(pic.PicError) as e:
        pic.pic_init_species(h, pic.species_desc(sp), 1)
    assert e.value.code == pic.PIC_EINVAL
    pic.pic_destroy(h)


def test_call_order_and_footprint():
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("sheet2d")
    h = pic.pic_create(pic.grid_desc(w))
    with pytest.raises(pic.PicError) as e:
        pic.pic_step(h, 1)
    assert e.value.code == pic.PIC_ESTATE
    sids = [pic.pic_init_species(h, pic.species_desc(sp), 1) for sp in w["species"]]
    assert [pic.pic_species_count(h, s) for s in sids] == [100 * 8, 100 * 10 * 4]
    fp = pic.pic_footprint(h)
    assert fp > 0 and fp == pic.pic_footprint(h)
    with pytest.raises(pic.PicError) as e:
        pic.pic_diag(h, pic.DIAG_FIELD_ENERGY)
    assert e.value.code == pic.PIC_ESTATE
    pic.pic_destroy(h)
    pic.pic_destroy(None)  # null-safe


def test_counts_match_oracle_loader(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    for name in ("slab1d", "disk2d", "sheet2d", "sphere3d"):
        w = W.small(name)
        h = pic.pic_create(pic.grid_desc(w))
        ref = oracle.build_workload(w)
        for sid, sp in enumerate(w["species"]):
            assert pic.pic_init_species(h, pic.species_desc(sp), 1) == sid
            assert pic.pic_species_count(h, sid) == ref.count(sid)
        pic.pic_destroy(h)
