"""Every device buffer of a filter context is released by glmb_destroy (CPU check of the
sources: the release list names each DevBuf member of the context and of its selection
buffers)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_06230_amd", "csrc")


def _members(text, start):
    k = text.index(start)
    body = text[k:text.index("};", k)]
    out = []
    for m in re.finditer(r"DevBuf ([^;]+);", body):
        out += [x.strip() for x in m.group(1).split(",") if x.strip()]
    return out


def test_destroy_releases_every_buffer():
    ctx = open(os.path.join(CSRC, "ctx.hpp")).read()
    common = open(os.path.join(CSRC, "common.hpp")).read()
    api = open(os.path.join(CSRC, "api.hip")).read()
    i = api.index("glmb::DevBuf* bufs[] = {")
    listed = api[i:api.index("};", i)]
    ctx_bufs = _members(ctx, "struct Ctx {")
    sb_bufs = _members(common, "struct SelectBufs")
    missing = [n for n in ctx_bufs if "&c.%s," % n not in listed and "&c.%s}" % n not in listed]
    missing += ["sb." + n for n in sb_bufs if "&c.sb.%s," % n not in listed and "&c.sb.%s}" % n not in listed]
    assert not missing, missing
